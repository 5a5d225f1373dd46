// lu.hip -- right-looking blocked LU without pivoting in mixed precision
// (paper: "Algorithmic Framework" and its Figure 1: the panel and the
// triangular solves in 32-bit, the Schur complement A22 - A21 A11^-1 A12 in
// 16-bit (or 8-bit) inputs with 32-bit accumulation; balancing/scaling of
// the input allowed).
//
// Per block step k (block size nb):
//   1. diagonal block A11 -> FP32, LU in FP32 with 64-wide inner blocking;
//      inverses of the 64x64 diagonal sub-blocks of L11 and U11 kept;
//   2. L21 = A21 U11^-1 and U12 = L11^-1 A12 by blocked substitution in
//      FP32, one workgroup per 32-row (32-column) strip, fused with the
//      rounding to the update format under a power-of-two strip scale;
//   3. A22 <- A22 - L21 U12 on the matrix cores (MFMA), FP32 accumulation,
//      result rounded to the storage format.
#include "common.hpp"
#include "kernels.hpp"

namespace mxp {

int dtype_bytes(int dt) {
    switch (dt) {
    case F64: return 8;
    case F32: return 4;
    case F16: case BF16: return 2;
    case F8: return 1;
    default: return 0;
    }
}

__host__ __device__ static inline int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

AuxLayout aux_layout(int64_t n, int64_t nb) {
    AuxLayout L;
    int64_t nblk = (n + nb - 1) / nb;
    size_t off = 0;
    L.T = off; off = al256(off + (size_t)nblk * nb * nb * 4);
    L.linv = off; off = al256(off + (size_t)nblk * nb * 64 * 4);
    L.uinv = off; off = al256(off + (size_t)nblk * nb * 64 * 4);
    L.lsc = off; off = al256(off + (size_t)nblk * ((n + 31) / 32) * 4);
    L.rowscale = off; off = al256(off + (size_t)n * 8);
    L.total = off;
    return L;
}

WorkLayout work_layout(int64_t n, int64_t nb, int update) {
    WorkLayout W;
    int64_t mpad = rup(n, 256);
    size_t eb = (size_t)dtype_bytes(update);
    size_t off = 0;
    W.Lq = off; off = al256(off + (size_t)mpad * nb * eb);
    W.Uq = off; off = al256(off + (size_t)mpad * nb * eb);
    W.inv_sa = off; off = al256(off + (size_t)(mpad / 32) * 4);
    W.inv_sb = off; off = al256(off + (size_t)(mpad / 32) * 4);
    W.info = off; off = al256(off + 8);
    W.total = off;
    return W;
}

// ============================================================== scaling
// Row equilibration: S_ii = 2^-p with 2^p the power of two nearest the
// diagonal (the largest entry of its row); A <- S A in place (exact except
// where a value drops into the subnormal range of the storage format).
template <int ST>
__global__ __launch_bounds__(256) void k_row_scale(int64_t n, typename Store<ST>::T* A, int64_t lda,
                                                   const double* __restrict__ diag, double* __restrict__ rowscale) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int e;
    double f = frexp(diag[i], &e);        // diag = f 2^e, f in [0.5, 1)
    int p = (f < 0.70710678118654752) ? e - 1 : e;
    double S = ldexp(1.0, -p);
    if (blockIdx.y == 0) rowscale[i] = S;
    float Sf = (float)S;
    int64_t j0 = (int64_t)blockIdx.y * 64;
    int64_t j1 = j0 + 64 < n ? j0 + 64 : n;
    for (int64_t j = j0; j < j1; ++j) {
        float v = Store<ST>::load(A, i + j * lda);
        A[i + j * lda] = Store<ST>::from_f32(v * Sf);
    }
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t row_equilibrate(const FactorPlan& p, const double* diag, hipStream_t s) {
    dim3 g((unsigned)((p.n + 255) / 256), (unsigned)((p.n + 63) / 64));
    switch (p.store) {
    case F32: k_row_scale<F32><<<g, 256, 0, s>>>(p.n, (float*)p.A, p.lda, diag, p.rowscale); break;
    case F16: k_row_scale<F16><<<g, 256, 0, s>>>(p.n, (half_t*)p.A, p.lda, diag, p.rowscale); break;
    case BF16: k_row_scale<BF16><<<g, 256, 0, s>>>(p.n, (bf16_t*)p.A, p.lda, diag, p.rowscale); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ============================================================== diagonal block
// T (FP32, ld = nb) <- A11, padded to a multiple of 64 with the identity.
template <int ST>
__global__ __launch_bounds__(256) void k_diag_load(const typename Store<ST>::T* A, int64_t lda, int64_t k, int kb,
                                                   int kbp, float* T, int ldt) {
    int j = blockIdx.y;
    for (int i = threadIdx.x; i < kbp; i += 256) {
        float v;
        if (i < kb && j < kb) v = Store<ST>::load(A, (k + i) + (k + j) * lda);
        else v = (i == j) ? 1.0f : 0.0f;
        T[i + (int64_t)j * ldt] = v;
    }
}

// A11 (storage format) <- T (FP32 L11\U11)
template <int ST>
__global__ __launch_bounds__(256) void k_diag_store(typename Store<ST>::T* A, int64_t lda, int64_t k, int kb,
                                                    const float* T, int ldt) {
    int j = blockIdx.y;
    for (int i = threadIdx.x; i < kb; i += 256)
        A[(k + i) + (k + j) * lda] = Store<ST>::from_f32(T[i + (int64_t)j * ldt]);
}

// LU of the 64x64 tile T[s:s+64, s:s+64] in LDS, then the inverses of its
// unit-lower and upper factors by column sweeps.  A zero or non-finite
// pivot records its 1-based global column in *info (atomic min).
__global__ __launch_bounds__(256) void k_leaf_lu(float* T, int ldt, int s, float* linv, float* uinv,
                                                 unsigned long long* info, int64_t col0) {
    __shared__ float a[64][65];
    __shared__ float xl[64][65];
    __shared__ float xu[64][65];
    int tid = threadIdx.x;
    for (int e = tid; e < 4096; e += 256) {
        int i = e & 63, j = e >> 6;
        a[i][j] = T[(s + i) + (int64_t)(s + j) * ldt];
        xl[i][j] = (i == j) ? 1.0f : 0.0f;
        xu[i][j] = (i == j) ? 1.0f : 0.0f;
    }
    __syncthreads();
    for (int j = 0; j < 64; ++j) {
        float p = a[j][j];
        if (tid == 0 && (p == 0.0f || !isfinite(p))) atomicMin(info, (unsigned long long)(col0 + s + j + 1));
        if (tid > j && tid < 64) a[tid][j] = a[tid][j] / p;
        __syncthreads();
        int w = 63 - j;  // trailing size
        for (int e = tid; e < w * w; e += 256) {
            int i = j + 1 + e % w, c = j + 1 + e / w;
            a[i][c] -= a[i][j] * a[j][c];
        }
        __syncthreads();
    }
    // inverse of unit-lower L: X = I; for t: rows i > t: X[i][:t+1] -= L[i][t] X[t][:t+1]
    // inverse of U: X = I; for t from 63 down: X[t][:] /= U[t][t]; rows i < t: X[i][:] -= U[i][t] X[t][:]
    for (int t = 0; t < 64; ++t) {
        int tu = 63 - t;
        if (tid < 64) xu[tu][tid] = xu[tu][tid] / a[tu][tu];
        __syncthreads();
        for (int e = tid; e < 64 * 64; e += 256) {
            int i = e >> 6, c = e & 63;
            if (i > t && c <= t) xl[i][c] -= a[i][t] * xl[t][c];
            if (i < tu && c >= tu) xu[i][c] -= a[i][tu] * xu[tu][c];
        }
        __syncthreads();
    }
    for (int e = tid; e < 4096; e += 256) {
        int i = e & 63, j = e >> 6;
        T[(s + i) + (int64_t)(s + j) * ldt] = a[i][j];
        linv[i + 64 * j] = xl[i][j];
        uinv[i + 64 * j] = xu[i][j];
    }
}

// 64x64x64 FP32 product on LDS tiles: each of 256 threads owns a 4x4 block
// (rows 4*(tid/16).., cols 4*(tid%16)..) of C += A B.
__device__ __forceinline__ void tile64_fma(const float (*sA)[65], const float (*sB)[65], float c[4][4], int tid) {
    int r0 = (tid >> 4) * 4, c0 = (tid & 15) * 4;
#pragma unroll 8
    for (int k = 0; k < 64; ++k) {
        float av[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) { av[q] = sA[r0 + q][k]; bv[q] = sB[k][c0 + q]; }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int u = 0; u < 4; ++u) c[q][u] = fmaf(av[q], bv[u], c[q][u]);
    }
}

// Inner step s: tiles T[I, s] <- T[I, s] Uinv_s (I > s) and T[s, J] <- Linv_s T[s, J] (J > s)
__global__ __launch_bounds__(256) void k_inner_trsm(float* T, int ldt, int s, int kbp, const float* linv,
                                                    const float* uinv) {
    __shared__ float sX[64][65];
    __shared__ float sI[64][65];
    int tid = threadIdx.x;
    int R = (kbp - s - 64) / 64;
    int w = blockIdx.x;
    bool lower = w < R;
    int t = s + 64 + 64 * (lower ? w : w - R);
    int64_t r0 = lower ? t : s, c0 = lower ? s : t;
    const float* inv = lower ? uinv : linv;
    for (int e = tid; e < 4096; e += 256) {
        int i = e & 63, j = e >> 6;
        sX[i][j] = T[(r0 + i) + (c0 + j) * ldt];
        sI[i][j] = inv[i + 64 * j];
    }
    __syncthreads();
    float c[4][4] = {};
    if (lower) tile64_fma(sX, sI, c, tid);  // X Uinv
    else tile64_fma(sI, sX, c, tid);        // Linv X
    int rr = (tid >> 4) * 4, cc = (tid & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) T[(r0 + rr + q) + (c0 + cc + u) * ldt] = c[q][u];
}

// Inner step s: T[I, J] -= T[I, s] T[s, J] for I, J > s
__global__ __launch_bounds__(256) void k_inner_update(float* T, int ldt, int s, int kbp) {
    __shared__ float sA[64][65];
    __shared__ float sB[64][65];
    int tid = threadIdx.x;
    int R = (kbp - s - 64) / 64;
    int I = s + 64 + 64 * (blockIdx.x % R), J = s + 64 + 64 * (blockIdx.x / R);
    for (int e = tid; e < 4096; e += 256) {
        int i = e & 63, j = e >> 6;
        sA[i][j] = T[(I + i) + (int64_t)(s + j) * ldt];
        sB[i][j] = T[(s + i) + (int64_t)(J + j) * ldt];
    }
    __syncthreads();
    float c[4][4] = {};
    tile64_fma(sA, sB, c, tid);
    int rr = (tid >> 4) * 4, cc = (tid & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) T[(I + rr + q) + (int64_t)(J + cc + u) * ldt] -= c[q][u];
}

// ============================================================== strip TRSMs + rounding
constexpr int SR = 32;  // rows (columns) per strip of L21 (U12) and per scale

// L21 strip: X (32 x nb) = A21[rows, :] U11^-1 by blocked substitution over
// 64-column blocks, X_J = (A_J - sum_{I<J} X_I U_IJ) Uinv_J; then
// amax -> power-of-two scales; writes the operand Lq (K-major, update
// format, scaled), the stored L21 (storage format, scaled) and the scales.
template <int ST, int OP>
__global__ __launch_bounds__(256) void k_trsm_L(typename Store<ST>::T* A, int64_t lda, int64_t n, int64_t k, int nb,
                                                const float* __restrict__ T, const float* __restrict__ uinv,
                                                typename Operand<OP>::T* Lq, float* inv_sa, float* lsc_blk) {
    extern __shared__ float smem[];
    const int SP = nb + 4;                  // row pitch of the strip
    float* S = smem;                        // [SR][SP]
    float (*sU)[65] = (float (*)[65])(smem + SR * SP);
    int tid = threadIdx.x;
    int w = blockIdx.x;
    int64_t r0 = k + nb + (int64_t)SR * w;  // first global row of the strip
    int64_t rv = n - r0;                    // valid rows
    if (rv > SR) rv = SR;
    if (rv < 0) rv = 0;
    // load (rows beyond n are zero)
    for (int e = tid; e < SR * nb; e += 256) {
        int ii = e % SR, c = e / SR;
        S[ii * SP + c] = (ii < rv) ? Store<ST>::load(A, (r0 + ii) + (k + c) * lda) : 0.0f;
    }
    __syncthreads();
    const int cc = tid & 63, rb = (tid >> 6) * 8;  // this thread: column cc, rows rb..rb+7
    const int nbk = nb / 64;
    for (int J = 0; J < nbk; ++J) {
        float acc[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[r] = S[(rb + r) * SP + J * 64 + cc];
        for (int I = 0; I < J; ++I) {
            for (int e = tid; e < 4096; e += 256) {
                int i = e & 63, j = e >> 6;
                sU[i][j] = T[(I * 64 + i) + (int64_t)(J * 64 + j) * nb];
            }
            __syncthreads();
            for (int kk = 0; kk < 64; ++kk) {
                float u = sU[kk][cc];
#pragma unroll
                for (int r = 0; r < 8; ++r) acc[r] = fmaf(-S[(rb + r) * SP + I * 64 + kk], u, acc[r]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) S[(rb + r) * SP + J * 64 + cc] = acc[r];
        for (int e = tid; e < 4096; e += 256) {
            int i = e & 63, j = e >> 6;
            sU[i][j] = uinv[(int64_t)J * 4096 + i + 64 * j];
        }
        __syncthreads();
        float y[8] = {};
        for (int kk = 0; kk < 64; ++kk) {
            float u = sU[kk][cc];
#pragma unroll
            for (int r = 0; r < 8; ++r) y[r] = fmaf(S[(rb + r) * SP + J * 64 + kk], u, y[r]);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) S[(rb + r) * SP + J * 64 + cc] = y[r];
        __syncthreads();
    }
    // amax of the strip
    __shared__ float red[4];
    float m = 0.0f;
    for (int e = tid; e < SR * nb; e += 256) m = fmaxf(m, fabsf(S[(e / nb) * SP + (e % nb)]));
    m = warp_maxf(m);
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    float amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    float s_op = Operand<OP>::scaled ? pow2_scale(amax, Operand<OP>::scale_exp) : 1.0f;
    float s_st = Store<ST>::scaled ? pow2_scale(amax, Store<ST>::scale_exp) : 1.0f;
    if (tid == 0) {
        inv_sa[w] = 1.0f / s_op;
        if (rv > 0) lsc_blk[r0 / SR] = s_st;
    }
    // operand, K-major: row (SR*w + ii) holds nb contiguous values
    for (int e = tid; e < SR * nb; e += 256) {
        int ii = e / nb, c = e % nb;
        Lq[((int64_t)SR * w + ii) * nb + c] = Operand<OP>::from_f32(S[ii * SP + c] * s_op);
    }
    // stored L21 (column-major, scaled)
    for (int e = tid; e < SR * nb; e += 256) {
        int ii = e % SR, c = e / SR;
        if (ii < rv) A[(r0 + ii) + (k + c) * lda] = Store<ST>::from_f32(S[ii * SP + c] * s_st);
    }
}

// U12 strip: Y (nb x 32) = L11^-1 A12[:, cols] by blocked substitution over
// 64-row blocks, Y_I = Linv_I (A_I - sum_{J<I} L_IJ Y_J); operand Uq
// (K-major: column j has nb contiguous values) scaled, stored U12 unscaled.
template <int ST, int OP>
__global__ __launch_bounds__(256) void k_trsm_U(typename Store<ST>::T* A, int64_t lda, int64_t n, int64_t k, int nb,
                                                const float* __restrict__ T, const float* __restrict__ linv,
                                                typename Operand<OP>::T* Uq, float* inv_sb) {
    extern __shared__ float smem[];
    const int SP = nb + 4;
    float* S = smem;                        // [SR cols][SP]: S[cc*SP + kk]
    float (*sL)[65] = (float (*)[65])(smem + SR * SP);
    int tid = threadIdx.x;
    int w = blockIdx.x;
    int64_t c0 = k + nb + (int64_t)SR * w;
    int64_t cv = n - c0;
    if (cv > SR) cv = SR;
    if (cv < 0) cv = 0;
    for (int e = tid; e < SR * nb; e += 256) {
        int kk = e % nb, cc = e / nb;
        S[cc * SP + kk] = (cc < cv) ? Store<ST>::load(A, (k + kk) + (c0 + cc) * lda) : 0.0f;
    }
    __syncthreads();
    const int kr = tid & 63, cb = (tid >> 6) * 8;  // row kr of the 64-block, columns cb..cb+7
    const int nbk = nb / 64;
    for (int I = 0; I < nbk; ++I) {
        float acc[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[r] = S[(cb + r) * SP + I * 64 + kr];
        for (int J = 0; J < I; ++J) {
            for (int e = tid; e < 4096; e += 256) {
                int i = e >> 6, j = e & 63;
                sL[i][j] = T[(I * 64 + i) + (int64_t)(J * 64 + j) * nb];
            }
            __syncthreads();
            for (int t = 0; t < 64; ++t) {
                float l = sL[kr][t];
#pragma unroll
                for (int r = 0; r < 8; ++r) acc[r] = fmaf(-l, S[(cb + r) * SP + J * 64 + t], acc[r]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) S[(cb + r) * SP + I * 64 + kr] = acc[r];
        for (int e = tid; e < 4096; e += 256) {
            int i = e >> 6, j = e & 63;
            sL[i][j] = linv[(int64_t)I * 4096 + i + 64 * j];
        }
        __syncthreads();
        float y[8] = {};
        for (int t = 0; t < 64; ++t) {
            float l = sL[kr][t];
#pragma unroll
            for (int r = 0; r < 8; ++r) y[r] = fmaf(l, S[(cb + r) * SP + I * 64 + t], y[r]);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) S[(cb + r) * SP + I * 64 + kr] = y[r];
        __syncthreads();
    }
    __shared__ float red[4];
    float m = 0.0f;
    for (int e = tid; e < SR * nb; e += 256) m = fmaxf(m, fabsf(S[(e / nb) * SP + (e % nb)]));
    m = warp_maxf(m);
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    float amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    float s_op = Operand<OP>::scaled ? pow2_scale(amax, Operand<OP>::scale_exp) : 1.0f;
    if (tid == 0) inv_sb[w] = 1.0f / s_op;
    for (int e = tid; e < SR * nb; e += 256) {
        int cc = e / nb, kk = e % nb;
        Uq[((int64_t)SR * w + cc) * nb + kk] = Operand<OP>::from_f32(S[cc * SP + kk] * s_op);
        if (cc < cv) A[(k + kk) + (c0 + cc) * lda] = Store<ST>::from_f32(S[cc * SP + kk]);
    }
}

// ============================================================== trailing update (MFMA)
// C (M x N, storage format, column-major) -= diag(inv_sa) (Lq Uq^T) diag(inv_sb)
// Lq: M x K (K-major), Uq: N x K (K-major), K = nb.
// Tile 256 x 256, 512 threads = 8 waves in a 2 (M) x 4 (N) grid, each wave
// 128 x 64 = 4 x 2 MFMA 32x32 blocks.  K advances 128 bytes per stage
// through two LDS buffers; a lane's fragment for one MFMA is a contiguous
// run of the K-major row.
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef int i4v __attribute__((ext_vector_type(4)));

template <int OP> struct Mfma;
template <> struct Mfma<F16> {
    static constexpr int KB = 32;  // bytes of a row consumed per instruction (16 halves)
    static MXP_DEV f16v run(const char* a, const char* b, f16v c) {
        h8v x = *(const h8v*)a, y = *(const h8v*)b;
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(x, y, c, 0, 0, 0);
    }
};
template <> struct Mfma<BF16> {
    static constexpr int KB = 32;
    static MXP_DEV f16v run(const char* a, const char* b, f16v c) {
        b8v x = *(const b8v*)a, y = *(const b8v*)b;
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, c, 0, 0, 0);
    }
};
template <> struct Mfma<F8> {
    static constexpr int KB = 64;  // 64 fp8 values
    static MXP_DEV f16v run(const char* a, const char* b, f16v c) {
        i4v a0 = *(const i4v*)a, a1 = *(const i4v*)(a + 16);
        i4v b0 = *(const i4v*)b, b1 = *(const i4v*)(b + 16);
        i8v x = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
        i8v y = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
        // formats 0/0 = fp8 e4m3 for both operands; E8M0 scales of 1.0
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x, y, c, 0, 0, 0, 0x7f7f7f7f, 0, 0x7f7f7f7f);
    }
};
template <> struct Mfma<F32> {
    static constexpr int KB = 8;   // 2 floats
    static MXP_DEV f16v run(const char* a, const char* b, f16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(*(const float*)a, *(const float*)b, c, 0, 0, 0);
    }
};

constexpr int GT = 256;           // tile edge
constexpr int GBK = 128;          // K bytes per stage
constexpr int GPITCH = GBK + 16;  // LDS row pitch in bytes (conflict-free 16-byte reads)
constexpr int GSTAGE = GT * GPITCH;

template <int OP, int ST>
__global__ __launch_bounds__(512) void k_gemm_update(typename Store<ST>::T* C, int64_t ldc, int64_t M, int64_t N,
                                                     int K, const char* __restrict__ Aq, const char* __restrict__ Bq,
                                                     const float* __restrict__ inv_sa,
                                                     const float* __restrict__ inv_sb, int tiles_m) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    char* sA = lds;                  // [2][GT][GPITCH]
    char* sB = lds + 2 * GSTAGE;     // [2][GT][GPITCH]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;     // 2 x 4 waves
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int64_t row0 = (int64_t)tm * GT, col0 = (int64_t)tn * GT;
    constexpr int eb = sizeof(typename Operand<OP>::T);
    const int64_t Kbytes = (int64_t)K * eb;
    const char* gA = Aq + row0 * Kbytes;
    const char* gB = Bq + col0 * Kbytes;
    const int nst = (int)(Kbytes / GBK);

    // each thread moves 4 16-byte chunks of A and 4 of B per stage
    i4v ra[4], rb[4];
    auto gload = [&](int st) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int ch = tid + q * 512;          // 0..2047
            int r = ch >> 3, cb = (ch & 7) * 16;
            ra[q] = *(const i4v*)(gA + (int64_t)r * Kbytes + (int64_t)st * GBK + cb);
            rb[q] = *(const i4v*)(gB + (int64_t)r * Kbytes + (int64_t)st * GBK + cb);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int ch = tid + q * 512;
            int r = ch >> 3, cb = (ch & 7) * 16;
            *(i4v*)(sA + buf * GSTAGE + r * GPITCH + cb) = ra[q];
            *(i4v*)(sB + buf * GSTAGE + r * GPITCH + cb) = rb[q];
        }
    };

    f16v acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    gload(0);
    sstore(0);
    __syncthreads();
    constexpr int KB = Mfma<OP>::KB;
    const int half = (lane >> 5) * (KB / 2);
    const int lr = lane & 31;
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) gload(st + 1);
        const char* a_base = sA + buf * GSTAGE + (wm * 128 + lr) * GPITCH + half;
        const char* b_base = sB + buf * GSTAGE + (wn * 64 + lr) * GPITCH + half;
#pragma unroll(OP == F8 ? 1 : GBK / KB)
        for (int ks = 0; ks < GBK / KB; ++ks) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = Mfma<OP>::run(a_base + a * 32 * GPITCH + ks * KB, b_base + b * 32 * GPITCH + ks * KB,
                                              acc[a][b]);
        }
        if (st + 1 < nst) sstore(buf ^ 1);
        __syncthreads();
    }
    // epilogue: lane holds, per 32x32 block, column lr and rows 8*(r/4) + 4*(lane/32) + r%4
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t rbase = row0 + wm * 128 + a * 32;
        const float sa = inv_sa[rbase / 32];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t col = col0 + wn * 64 + b * 32 + lr;
            if (col >= N) continue;
            const float d = sa * inv_sb[(col0 + wn * 64 + b * 32) / 32];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t r = rbase + 8 * g + 4 * (lane >> 5);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (r + q < M) {
                        int64_t idx = (r + q) + col * ldc;
                        float v = Store<ST>::load(C, idx);
                        C[idx] = Store<ST>::from_f32(v - acc[a][b][g * 4 + q] * d);
                    }
                }
            }
        }
    }
}

// ============================================================== driver
static size_t trsm_smem(int nb) { return (size_t)(SR * (nb + 4) + 64 * 65) * sizeof(float); }

template <int ST, int OP>
static hipError_t factor_typed(const FactorPlan& p, hipStream_t s) {
    typedef typename Store<ST>::T ST_T;
    typedef typename Operand<OP>::T OP_T;
    static bool attr_done = false;
    hipError_t e;
    if (!attr_done) {
        if ((e = hipFuncSetAttribute((const void*)k_trsm_L<ST, OP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)trsm_smem(1024)))) return e;
        if ((e = hipFuncSetAttribute((const void*)k_trsm_U<ST, OP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)trsm_smem(1024)))) return e;
        if ((e = hipFuncSetAttribute((const void*)k_gemm_update<OP, ST>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     4 * GSTAGE))) return e;
        attr_done = true;
    }
    ST_T* A = (ST_T*)p.A;
    const int64_t n = p.n, lda = p.lda;
    const int nb = (int)p.nb;
    const int64_t nstrips_total = (n + SR - 1) / SR;
    if ((e = fill_u64(p.info, 1, ~0ull, s))) return e;
    for (int64_t k = 0; k < n; k += nb) {
        const int kb = (int)(n - k < nb ? n - k : nb);
        const int kbp = (int)rup(kb, 64);
        const int64_t m = n - k - kb;
        const int64_t blk = k / nb;
        float* T = p.T + blk * nb * nb;
        float* linv = p.linv + blk * nb * 64;
        float* uinv = p.uinv + blk * nb * 64;
        k_diag_load<ST><<<dim3(1, kbp), 256, 0, s>>>(A, lda, k, kb, kbp, T, nb);
        for (int sb = 0; sb < kbp; sb += 64) {
            k_leaf_lu<<<1, 256, 0, s>>>(T, nb, sb, linv + (sb / 64) * 4096, uinv + (sb / 64) * 4096, p.info, k);
            if (sb + 64 < kbp) {
                int R = (kbp - sb - 64) / 64;
                k_inner_trsm<<<2 * R, 256, 0, s>>>(T, nb, sb, kbp, linv + (sb / 64) * 4096, uinv + (sb / 64) * 4096);
                k_inner_update<<<R * R, 256, 0, s>>>(T, nb, sb, kbp);
            }
        }
        k_diag_store<ST><<<dim3(1, kb), 256, 0, s>>>(A, lda, k, kb, T, nb);
        if ((e = hipGetLastError())) return e;
        if (m > 0) {
            const int nstrip = (int)(rup(m, GT) / SR);
            const size_t smem = trsm_smem(nb);
            k_trsm_L<ST, OP><<<nstrip, 256, smem, s>>>(A, lda, n, k, nb, T, uinv, (OP_T*)p.Lq, p.inv_sa,
                                                       p.lsc + blk * nstrips_total);
            k_trsm_U<ST, OP><<<nstrip, 256, smem, s>>>(A, lda, n, k, nb, T, linv, (OP_T*)p.Uq, p.inv_sb);
            const int tiles = (int)((m + GT - 1) / GT);
            ST_T* C = A + (k + kb) + (k + kb) * lda;
            k_gemm_update<OP, ST><<<tiles * tiles, 512, 4 * GSTAGE, s>>>(C, lda, m, m, nb, (const char*)p.Lq,
                                                                         (const char*)p.Uq, p.inv_sa, p.inv_sb, tiles);
            if ((e = hipGetLastError())) return e;
        }
    }
    return hipSuccess;
}

hipError_t factor_run(const FactorPlan& p, hipStream_t s) {
    const int u = p.update, t = p.store;
    if (u == F32 && t == F32) return factor_typed<F32, F32>(p, s);
    if (u == F16 && t == F16) return factor_typed<F16, F16>(p, s);
    if (u == BF16 && t == BF16) return factor_typed<BF16, BF16>(p, s);
    if (u == F8 && t == F16) return factor_typed<F16, F8>(p, s);
    if (u == F8 && t == BF16) return factor_typed<BF16, F8>(p, s);
    if (u == F16 && t == F32) return factor_typed<F32, F16>(p, s);
    if (u == BF16 && t == F32) return factor_typed<F32, BF16>(p, s);
    return hipErrorInvalidValue;
}

}  // namespace mxp
