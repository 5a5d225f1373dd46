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
#include "prof.hpp"

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
    L.Trm = off; off = al256(off + (size_t)nblk * nb * nb * 4);
    L.linv = off; off = al256(off + (size_t)nblk * nb * 64 * 4);
    L.uinv = off; off = al256(off + (size_t)nblk * nb * 64 * 4);
    L.lsc = off; off = al256(off + (size_t)nblk * ((n + 31) / 32) * 4);
    L.rowscale = off; off = al256(off + (size_t)n * 8);
    L.linv_full = off; off = al256(off + (size_t)nblk * nb * nb * 4);
    L.uinv_full = off; off = al256(off + (size_t)nblk * nb * nb * 4);
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

// A11 (storage format) <- T (FP32 L11\U11); Trm <- T transposed (row-major
// copy: rows of U11 contiguous), padded part included.
template <int ST>
__global__ __launch_bounds__(256) void k_diag_store(typename Store<ST>::T* A, int64_t lda, int64_t k, int kb, int kbp,
                                                    const float* T, float* Trm, int ldt) {
    __shared__ float tile[64][65];
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
    for (int c = g; c < 64; c += 4) {
        const float v = T[(i0 + r) + (int64_t)(j0 + c) * ldt];
        tile[r][c] = v;
        if (i0 + r < kb && j0 + c < kb) A[(k + i0 + r) + (k + j0 + c) * lda] = Store<ST>::from_f32(v);
    }
    __syncthreads();
    for (int c = g; c < 64; c += 4) Trm[(j0 + r) + (int64_t)(i0 + c) * ldt] = tile[c][r];
}

// LU of the 64x64 tile T[s:s+64, s:s+64] in LDS, then the inverses of its
// unit-lower and upper factors by column sweeps (L^-1 stored column-major,
// U^-1 row-major: both are then read along contiguous runs by the MFMA
// operand loads of the strip solves).  Thread (r, g): row r,
// columns g, g+4, ...  A zero or non-finite pivot records its 1-based
// global column in *info (atomic min).
__global__ __launch_bounds__(256) void k_leaf_lu(float* T, int ldt, int s, float* linv, float* uinv,
                                                 unsigned long long* info, int64_t col0) {
    __shared__ float a[64][65];
    __shared__ float xl[64][65];
    __shared__ float xu[64][65];
    const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
    for (int c = g; c < 64; c += 4) {
        a[r][c] = T[(s + r) + (int64_t)(s + c) * ldt];
        xl[r][c] = (r == c) ? 1.0f : 0.0f;
        xu[r][c] = (r == c) ? 1.0f : 0.0f;
    }
    __syncthreads();
    for (int j = 0; j < 64; ++j) {
        const float p = a[j][j];
        if (tid == 0 && (p == 0.0f || !isfinite(p))) atomicMin(info, (unsigned long long)(col0 + s + j + 1));
        if (g == 0 && r > j) a[r][j] = a[r][j] / p;
        __syncthreads();
        if (r > j) {
            const float l = a[r][j];
            for (int c = j + 1 + g; c < 64; c += 4) a[r][c] -= l * a[j][c];
        }
        __syncthreads();
    }
    // L^-1: X = I; for t ascending, rows i > t: X[i][0:t] -= L[i][t] X[t][0:t]
    // U^-1: X = I; for t descending: X[t][:] /= U[t][t]; rows i < t: X[i][t:] -= U[i][t] X[t][t:]
    for (int t = 0; t < 64; ++t) {
        const int tu = 63 - t;
        if (g == 0) xu[tu][r] = xu[tu][r] / a[tu][tu];
        __syncthreads();
        if (r > t) {
            const float l = a[r][t];
            for (int c = g; c <= t; c += 4) xl[r][c] -= l * xl[t][c];
        }
        if (r < tu) {
            const float u = a[r][tu];
            for (int c = tu + g; c < 64; c += 4) xu[r][c] -= u * xu[tu][c];
        }
        __syncthreads();
    }
    for (int c = g; c < 64; c += 4) {
        T[(s + r) + (int64_t)(s + c) * ldt] = a[r][c];
        linv[r + 64 * c] = xl[r][c];
        uinv[64 * r + c] = xu[r][c];   // row-major (U^-1 read by rows)
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
    for (int e = tid; e < 4096; e += 256) {
        int i = e & 63, j = e >> 6;
        sX[i][j] = T[(r0 + i) + (c0 + j) * ldt];
        sI[i][j] = lower ? uinv[64 * i + j] : linv[i + 64 * j];
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

// The strip solves run on the FP32 matrix cores (v_mfma_f32_32x32x2f32):
// lane l holds A[l%32][k0 + l/32] and B[k0 + l/32][l%32]; the 32x32 result
// sits in 16 registers, register q of lane l being row 8(q/4) + 4(l/32) + q%4,
// column l%32.  The strip lives in LDS (pitch odd, so the 32 rows / columns
// a fragment touches fall in distinct banks); the factor blocks stream from
// L2 straight into operand registers along contiguous runs.
typedef float f16v_t __attribute__((ext_vector_type(16)));

MXP_DEV f16v_t mfma2(float a, float b, f16v_t c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }

// add the other K-half's partial results (waves 2,3 -> waves 0,1) through LDS
MXP_DEV void khalf_reduce(f16v_t& acc, float* red, int blk, int kh, int lane) {
    if (kh == 1)
        for (int q = 0; q < 16; ++q) red[(blk * 16 + q) * 64 + lane] = acc[q];
    __syncthreads();
    if (kh == 0)
        for (int q = 0; q < 16; ++q) acc[q] += red[(blk * 16 + q) * 64 + lane];
}

// Right solve of a 32-row strip S (row i at S + i*SP): X <- S U^-1 block by
// block, X_J = (S_J - sum_{I<J} X_I U_IJ) Uinv_J.  Urm: U11 row-major (ld),
// uinv_rm: the 64x64 diagonal-block inverses, row-major.
__device__ void strip_right_solve(float* S, int SP, int nbk, const float* __restrict__ Urm, int ld,
                                  const float* __restrict__ uinv_rm, float* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 31, lh = lane >> 5, blk = wave & 1, kh = wave >> 1;
    for (int J = 0; J < nbk; ++J) {
        const int jc = J * 64 + blk * 32 + lr;            // this lane's column of the output block
        f16v_t acc = {};
        for (int I = 0; I < J; ++I) {
            const int kb0 = I * 64 + kh * 32 + lh;
            float bv[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) bv[s2] = Urm[(int64_t)(kb0 + 2 * s2) * ld + jc];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) acc = mfma2(S[lr * SP + kb0 + 2 * s2], bv[s2], acc);
        }
        khalf_reduce(acc, red, blk, kh, lane);
        if (kh == 0)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = 8 * (q >> 2) + 4 * lh + (q & 3);
                S[i * SP + jc] -= acc[q];
            }
        __syncthreads();
        f16v_t y = {};
        {
            const int k0 = kh * 32 + lh;
            float bv[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) bv[s2] = uinv_rm[(int64_t)J * 4096 + (k0 + 2 * s2) * 64 + blk * 32 + lr];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) y = mfma2(S[lr * SP + J * 64 + k0 + 2 * s2], bv[s2], y);
        }
        khalf_reduce(y, red, blk, kh, lane);
        if (kh == 0)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = 8 * (q >> 2) + 4 * lh + (q & 3);
                S[i * SP + jc] = y[q];
            }
        __syncthreads();
    }
}

// Left solve of a 32-column strip S (column j at S + j*SP): Y <- L^-1 S,
// Y_I = Linv_I (S_I - sum_{J<I} L_IJ Y_J).  T: L11 column-major (ld),
// linv: the 64x64 diagonal-block inverses, column-major.
__device__ void strip_left_solve(float* S, int SP, int nbk, const float* __restrict__ T, int ld,
                                 const float* __restrict__ linv, float* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 31, lh = lane >> 5, blk = wave & 1, kh = wave >> 1;
    for (int I = 0; I < nbk; ++I) {
        const int ir = I * 64 + blk * 32 + lr;            // this lane's row of L for the A operand
        f16v_t acc = {};
        for (int J = 0; J < I; ++J) {
            const int kb0 = J * 64 + kh * 32 + lh;
            float av[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) av[s2] = T[ir + (int64_t)(kb0 + 2 * s2) * ld];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) acc = mfma2(av[s2], S[lr * SP + kb0 + 2 * s2], acc);
        }
        khalf_reduce(acc, red, blk, kh, lane);
        if (kh == 0)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = I * 64 + blk * 32 + 8 * (q >> 2) + 4 * lh + (q & 3);
                S[lr * SP + i] -= acc[q];
            }
        __syncthreads();
        f16v_t y = {};
        {
            const int k0 = kh * 32 + lh;
            float av[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) av[s2] = linv[(int64_t)I * 4096 + (blk * 32 + lr) + 64 * (k0 + 2 * s2)];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) y = mfma2(av[s2], S[lr * SP + I * 64 + k0 + 2 * s2], y);
        }
        khalf_reduce(y, red, blk, kh, lane);
        if (kh == 0)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = I * 64 + blk * 32 + 8 * (q >> 2) + 4 * lh + (q & 3);
                S[lr * SP + i] = y[q];
            }
        __syncthreads();
    }
}

__device__ float strip_amax(const float* S, int SP, int width) {
    __shared__ float red[4];
    const int tid = threadIdx.x;
    float m = 0.0f;
    for (int e = tid; e < SR * width; e += 256) m = fmaxf(m, fabsf(S[(e / width) * SP + (e % width)]));
    m = warp_maxf(m);
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    float amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    return amax;
}

// LDS of a strip kernel: the strip (32 x (nb+1) floats) and the K-half reduction buffer
static inline size_t trsm_smem(int nb) { return (size_t)(SR * (nb + 1) + 2 * 16 * 64) * sizeof(float); }

// L21 strip: X (32 x nb) = A21[rows, :] U11^-1, then amax -> power-of-two
// scales; writes the operand Lq (K-major, update format, scaled), the stored
// L21 (storage format, scaled) and the scales.
template <int ST, int OP>
__global__ __launch_bounds__(256) void k_trsm_L(typename Store<ST>::T* A, int64_t lda, int64_t n, int64_t k, int nb,
                                                const float* __restrict__ Urm, const float* __restrict__ uinv,
                                                typename Operand<OP>::T* Lq, float* inv_sa, float* lsc_blk) {
    extern __shared__ float smem[];
    const int SP = nb + 1;
    float* S = smem;
    float* red = smem + SR * SP;
    const int tid = threadIdx.x, w = blockIdx.x;
    const int64_t r0 = k + nb + (int64_t)SR * w;
    int64_t rv = n - r0;
    rv = rv > SR ? SR : (rv < 0 ? 0 : rv);
    for (int e = tid; e < SR * nb; e += 256) {
        int ii = e % SR, c = e / SR;
        S[ii * SP + c] = (ii < rv) ? Store<ST>::load(A, (r0 + ii) + (k + c) * lda) : 0.0f;
    }
    __syncthreads();
    strip_right_solve(S, SP, nb / 64, Urm, nb, uinv, red);
    const float amax = strip_amax(S, SP, nb);
    const float s_op = Operand<OP>::scaled ? pow2_scale(amax, Operand<OP>::scale_exp) : 1.0f;
    const float s_st = Store<ST>::scaled ? pow2_scale(amax, Store<ST>::scale_exp) : 1.0f;
    if (tid == 0) {
        inv_sa[w] = 1.0f / s_op;
        if (rv > 0) lsc_blk[r0 / SR] = s_st;
    }
    for (int e = tid; e < SR * nb; e += 256) {
        int ii = e / nb, c = e % nb;
        Lq[((int64_t)SR * w + ii) * nb + c] = Operand<OP>::from_f32(S[ii * SP + c] * s_op);
    }
    for (int e = tid; e < SR * nb; e += 256) {
        int ii = e % SR, c = e / SR;
        if (ii < rv) A[(r0 + ii) + (k + c) * lda] = Store<ST>::from_f32(S[ii * SP + c] * s_st);
    }
}

// U12 strip: Y (nb x 32) = L11^-1 A12[:, cols]; operand Uq (K-major: column
// j has nb contiguous values) scaled, stored U12 unscaled.
template <int ST, int OP>
__global__ __launch_bounds__(256) void k_trsm_U(typename Store<ST>::T* A, int64_t lda, int64_t n, int64_t k, int nb,
                                                const float* __restrict__ T, const float* __restrict__ linv,
                                                typename Operand<OP>::T* Uq, float* inv_sb) {
    extern __shared__ float smem[];
    const int SP = nb + 1;
    float* S = smem;
    float* red = smem + SR * SP;
    const int tid = threadIdx.x, w = blockIdx.x;
    const int64_t c0 = k + nb + (int64_t)SR * w;
    int64_t cv = n - c0;
    cv = cv > SR ? SR : (cv < 0 ? 0 : cv);
    for (int e = tid; e < SR * nb; e += 256) {
        int kk = e % nb, cc = e / nb;
        S[cc * SP + kk] = (cc < cv) ? Store<ST>::load(A, (k + kk) + (c0 + cc) * lda) : 0.0f;
    }
    __syncthreads();
    strip_left_solve(S, SP, nb / 64, T, nb, linv, red);
    const float amax = strip_amax(S, SP, nb);
    const float s_op = Operand<OP>::scaled ? pow2_scale(amax, Operand<OP>::scale_exp) : 1.0f;
    if (tid == 0) inv_sb[w] = 1.0f / s_op;
    for (int e = tid; e < SR * nb; e += 256) {
        int cc = e / nb, kk = e % nb;
        Uq[((int64_t)SR * w + cc) * nb + kk] = Operand<OP>::from_f32(S[cc * SP + kk] * s_op);
        if (cc < cv) A[(k + kk) + (c0 + cc) * lda] = Store<ST>::from_f32(S[cc * SP + kk]);
    }
}

// Full inverses of the diagonal blocks (for the preconditioner), all blocks
// in one launch: blockIdx.y = block, blockIdx.x = 32-wide strip.
// U11^-1 rows r0..r0+31 = I[r0:r0+32, :] U11^-1; L11^-1 columns = L11^-1 I[:, c0:c0+32].
__global__ __launch_bounds__(256) void k_inv_upper(int64_t n, int nb, const float* __restrict__ Trm_all,
                                                   const float* __restrict__ uinv_all, float* __restrict__ out_all) {
    extern __shared__ float smem[];
    const int64_t blk = blockIdx.y;
    const int64_t k = blk * nb;
    const int kb = (int)(n - k < nb ? n - k : nb);
    const int kbp = (kb + 63) / 64 * 64;
    const int r0 = SR * blockIdx.x;
    if (r0 >= kbp) return;
    const int SP = kbp + 1;
    float* S = smem;
    float* red = smem + SR * SP;
    for (int e = threadIdx.x; e < SR * kbp; e += 256) {
        int ii = e % SR, c = e / SR;
        S[ii * SP + c] = (r0 + ii == c) ? 1.0f : 0.0f;
    }
    __syncthreads();
    strip_right_solve(S, SP, kbp / 64, Trm_all + blk * nb * nb, nb, uinv_all + blk * nb * 64, red);
    float* out = out_all + blk * nb * nb;
    for (int e = threadIdx.x; e < SR * kbp; e += 256) {
        int ii = e % SR, c = e / SR;
        out[(r0 + ii) + (int64_t)c * nb] = S[ii * SP + c];
    }
}

__global__ __launch_bounds__(256) void k_inv_lower(int64_t n, int nb, const float* __restrict__ Tall,
                                                   const float* __restrict__ linv_all, float* __restrict__ out_all) {
    extern __shared__ float smem[];
    const int64_t blk = blockIdx.y;
    const int64_t k = blk * nb;
    const int kb = (int)(n - k < nb ? n - k : nb);
    const int kbp = (kb + 63) / 64 * 64;
    const int c0 = SR * blockIdx.x;
    if (c0 >= kbp) return;
    const int SP = kbp + 1;
    float* S = smem;
    float* red = smem + SR * SP;
    for (int e = threadIdx.x; e < SR * kbp; e += 256) {
        int kk = e % kbp, cc = e / kbp;
        S[cc * SP + kk] = (kk == c0 + cc) ? 1.0f : 0.0f;
    }
    __syncthreads();
    strip_left_solve(S, SP, kbp / 64, Tall + blk * nb * nb, nb, linv_all + blk * nb * 64, red);
    float* out = out_all + blk * nb * nb;
    for (int e = threadIdx.x; e < SR * kbp; e += 256) {
        int kk = e % kbp, cc = e / kbp;
        out[kk + (int64_t)(c0 + cc) * nb] = S[cc * SP + kk];
    }
}

// ============================================================== driver

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
        if ((e = hipFuncSetAttribute((const void*)k_inv_upper, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)trsm_smem(1024)))) return e;
        if ((e = hipFuncSetAttribute((const void*)k_inv_lower, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)trsm_smem(1024)))) return e;
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
        prof::begin(s);
        k_diag_load<ST><<<dim3(1, kbp), 256, 0, s>>>(A, lda, k, kb, kbp, T, nb);
        for (int sb = 0; sb < kbp; sb += 64) {
            k_leaf_lu<<<1, 256, 0, s>>>(T, nb, sb, linv + (sb / 64) * 4096, uinv + (sb / 64) * 4096, p.info, k);
            if (sb + 64 < kbp) {
                int R = (kbp - sb - 64) / 64;
                k_inner_trsm<<<2 * R, 256, 0, s>>>(T, nb, sb, kbp, linv + (sb / 64) * 4096, uinv + (sb / 64) * 4096);
                k_inner_update<<<R * R, 256, 0, s>>>(T, nb, sb, kbp);
            }
        }
        k_diag_store<ST><<<dim3(kbp / 64, kbp / 64), 256, 0, s>>>(A, lda, k, kb, kbp, T, p.Trm + blk * nb * nb, nb);
        prof::end(prof::DIAG, s, 2.0 / 3.0 * kb * (double)kb * kb, 2.0 * kb * (double)kb * sizeof(ST_T));
        if ((e = hipGetLastError())) return e;
        if (m > 0) {
            const int nstrip = (int)(rup(m, 256) / SR);
            const size_t smem = trsm_smem(nb);
            prof::begin(s);
            k_trsm_L<ST, OP><<<nstrip, 256, smem, s>>>(A, lda, n, k, nb, p.Trm + blk * nb * nb, uinv, (OP_T*)p.Lq, p.inv_sa,
                                                       p.lsc + blk * nstrips_total);
            k_trsm_U<ST, OP><<<nstrip, 256, smem, s>>>(A, lda, n, k, nb, T, linv, (OP_T*)p.Uq, p.inv_sb);
            prof::end(prof::TRSM, s, 2.0 * m * (double)nb * nb,
                      4.0 * m * (double)nb * sizeof(ST_T) + 2.0 * m * (double)nb * sizeof(OP_T));
            prof::begin(s);
            ST_T* C = A + (k + kb) + (k + kb) * lda;
            if ((e = gemm_update(OP, ST, C, lda, m, m, nb, p.Lq, p.Uq, p.inv_sa, p.inv_sb, s))) return e;
            prof::end(prof::GEMM, s, 2.0 * m * (double)m * nb,
                      2.0 * m * (double)m * sizeof(ST_T) + 2.0 * m * (double)nb * sizeof(OP_T));
            if ((e = hipGetLastError())) return e;
        }
    }
    // full FP32 inverses of every diagonal block, used by the preconditioner
    {
        const int64_t nblk = (n + nb - 1) / nb;
        dim3 g((unsigned)(nb / SR), (unsigned)nblk);
        prof::begin(s);
        k_inv_upper<<<g, 256, trsm_smem(nb), s>>>(n, nb, p.Trm, p.uinv, p.uinv_full);
        k_inv_lower<<<g, 256, trsm_smem(nb), s>>>(n, nb, p.T, p.linv, p.linv_full);
        prof::end(prof::DIAG, s, 2.0 / 3.0 * (double)n * nb * nb, 16.0 * (double)n * nb);
        if ((e = hipGetLastError())) return e;
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
