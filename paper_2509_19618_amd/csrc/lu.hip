// lu.hip -- right-looking blocked LU without pivoting in mixed precision
// (paper: "Algorithmic Framework" and its Figure 1: the panel and the
// triangular solves in 32-bit, the Schur complement A22 - A21 A11^-1 A12 in
// 16-bit (or 8-bit) inputs with 32-bit accumulation; balancing/scaling of
// the input allowed).
//
// Per block step k (block size nb):
//   1. diagonal block A11 -> FP32, LU in FP32 by up to 24 cooperating
//      work-groups over 32x32 tiles (diag.hip); inverses of the 64x64
//      diagonal sub-blocks of L11 and U11 kept;
//   2. L21 = A21 U11^-1 and U12 = L11^-1 A12 by blocked substitution in
//      FP32, one workgroup per 32-row (32-column) strip, fused with the
//      rounding to the update format under a power-of-two strip scale;
//   3. A22 <- A22 - L21 U12 on the matrix cores (MFMA), FP32 accumulation,
//      result rounded to the storage format.
#include <mutex>
#include <vector>

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
    const int64_t D = prec_block(nb), ngrp = (n + D - 1) / D;
    L.linv_full = off; off = al256(off + (size_t)ngrp * D * D * 4);
    L.uinv_full = off; off = al256(off + (size_t)ngrp * D * D * 4);
    L.total = off;
    return L;
}

// operand rows per set: the trailing size padded to 256, plus 256 so that
// the sub-range updates of the look-ahead (starting nb rows in) stay inside
int64_t operand_rows(int64_t n) { return rup(n, 256) + 256; }

WorkLayout work_layout(int64_t n, int64_t nb, int update) {
    WorkLayout W;
    int64_t rows = operand_rows(n);
    size_t eb = (size_t)dtype_bytes(update);
    size_t off = 0;
    W.Lq = off; off = al256(off + 4 * (size_t)rows * nb * eb);     // four sets: two pairs of steps
    W.Uq = off; off = al256(off + 4 * (size_t)rows * nb * eb);
    W.inv_sa = off; off = al256(off + 4 * (size_t)(rows / 32) * 4);
    W.inv_sb = off; off = al256(off + 4 * (size_t)(rows / 32) * 4);
    W.info = off; off = al256(off + 8);
    W.dsync = off; off = al256(off + (size_t)((n + nb - 1) / nb) * diag_sync_words() * 4);
    W.pairw = off;
    if (prec_block(nb) == 2 * nb) off = al256(off + (size_t)((n + 2 * nb - 1) / (2 * nb)) * nb * nb * 4);
    W.binv = off; off = al256(off + (size_t)2 * 3 * nb * nb * 2);
    W.binv_sc = off; off = al256(off + (size_t)2 * nb * 4);
    W.total = off;
    return W;
}

// ============================================================== scaling
// Row equilibration: S_ii = 2^(t - p) with 2^p the power of two nearest the
// diagonal (the largest entry of its row), so the diagonal lands near 2^t;
// A <- S A in place, exactly.  t = 14 for FP16 storage, whose normal range
// ends below 2^-14: with the diagonal near 1 the off-diagonal entries (about
// n/4 times smaller) would be stored as subnormals, with the diagonal near
// 2^14 they stay normal; t = 0 for BF16 and FP32 storage.
template <int ST>
__global__ __launch_bounds__(256) void k_row_scale(int64_t n, typename Store<ST>::T* A, int64_t lda,
                                                   const double* __restrict__ diag, double* __restrict__ rowscale,
                                                   int target) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int e;
    double f = frexp(diag[i], &e);        // diag = f 2^e, f in [0.5, 1)
    int p = (f < 0.70710678118654752) ? e - 1 : e;
    double S = ldexp(1.0, target - p);
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
    case F32: k_row_scale<F32><<<g, 256, 0, s>>>(p.n, (float*)p.A, p.lda, diag, p.rowscale, 0); break;
    case F16: k_row_scale<F16><<<g, 256, 0, s>>>(p.n, (half_t*)p.A, p.lda, diag, p.rowscale, 14); break;
    case BF16: k_row_scale<BF16><<<g, 256, 0, s>>>(p.n, (bf16_t*)p.A, p.lda, diag, p.rowscale, 0); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ============================================================== strip TRSMs + rounding
typedef float f16v_t __attribute__((ext_vector_type(16)));
MXP_DEV f16v_t mfma2(float a, float b, f16v_t c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }

constexpr int SR = 32;  // rows (columns) per strip of L21 (U12) and per scale

// The strip solves run on the FP32 matrix cores (v_mfma_f32_32x32x2f32):
// lane l holds A[l%32][k0 + l/32] and B[k0 + l/32][l%32]; the 32x32 result
// sits in 16 registers, register q of lane l being row 8(q/4) + 4(l/32) + q%4,
// column l%32.  The strip lives in LDS (pitch odd, so the 32 rows / columns
// a fragment touches fall in distinct banks); the factor blocks stream from
// L2 straight into operand registers along contiguous runs.
// v, treated as written here: a batch of LDS reads feeding an MFMA chain
// completes before the chain (one wait), instead of one wait per product
MXP_DEV void pin_f(float& v) { asm volatile("" : "+v"(v)); }

// add the other K-half's partial results (waves 2,3 -> waves 0,1) through LDS
MXP_DEV void khalf_reduce(f16v_t& acc, float* red, int blk, int kh, int lane) {
    if (kh == 1)
        for (int q = 0; q < 16; ++q) red[(blk * 16 + q) * 64 + lane] = acc[q];
    __syncthreads();
    if (kh == 0)
        for (int q = 0; q < 16; ++q) acc[q] += red[(blk * 16 + q) * 64 + lane];
}

// maximum of v over the work-group (red: at least 4 floats of LDS, free)
MXP_DEV float strip_max(float v, float* red) {
    v = warp_maxf(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const float r = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    __syncthreads();
    return r;
}

// four consecutive elements of a storage or operand array, one access
template <class T> struct alignas(4 * sizeof(T)) Pack4 {
    T v[4];
};

// Right solve of a 32-row strip S (row i at S + i*SP): X <- S U^-1 block by
// block, X_J = (S_J - sum_{I<J} X_I U_IJ) Uinv_J.  Urm: U11 row-major (ld),
// uinv_rm: the 64x64 diagonal-block inverses, row-major.  The factor blocks
// do not depend on the strip: block I+1 is loaded while block I is applied,
// and the first block and the inverse block of step J+1 are loaded while
// step J finishes (its reductions and inverse product), so that a step
// never starts with a load latency.
MXP_DEV float strip_right_solve(float* S, int SP, int nbk, const float* __restrict__ Urm, int ld,
                                   const float* __restrict__ uinv_rm, float* red) {
    float m = 0.0f;   // max |x| over this lane's final stores
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 31, lh = lane >> 5, blk = wave & 1, kh = wave >> 1;
    const int k0 = kh * 32 + lh;
    auto ld_iv = [&](float* v, int J) {
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) v[s2] = uinv_rm[(int64_t)J * 4096 + (k0 + 2 * s2) * 64 + blk * 32 + lr];
    };
    // a block's sixteen loads: a wave-uniform base (kept in scalar
    // registers) plus one 32-bit lane offset
    const int ld2 = 2 * ld;
    auto ld_blk = [&](float* bv, int I, int J) {
        const float* ub = Urm + (int64_t)(I * 64 + kh * 32) * ld + J * 64 + blk * 32;
        const int lo = lh * ld + lr;
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) bv[s2] = ub[s2 * ld2 + lo];
    };
    float iv[16], ivn[16], b0[16], b1[16];
    ld_iv(iv, 0);
    for (int J = 0; J < nbk; ++J) {
        const int jc = J * 64 + blk * 32 + lr;            // this lane's column of the output block
        f16v_t acc = {};
        auto mf_blk = [&](const float* bv, int I) {
            const int kb0 = I * 64 + k0;
            float av[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) av[s2] = S[lr * SP + kb0 + 2 * s2];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) pin_f(av[s2]);
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) acc = mfma2(av[s2], bv[s2], acc);
        };
        // b0 holds block (0, J) for J > 0 (loaded during step J - 1)
        int I = 0;
        for (; I + 1 < J; I += 2) {
            ld_blk(b1, I + 1, J);
            mf_blk(b0, I);
            if (I + 2 < J) ld_blk(b0, I + 2, J);
            mf_blk(b1, I + 1);
        }
        if (I < J) mf_blk(b0, I);
        if (J + 1 < nbk) {
            ld_blk(b0, 0, J + 1);
            ld_iv(ivn, J + 1);
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
            float av[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) av[s2] = S[lr * SP + J * 64 + k0 + 2 * s2];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) pin_f(av[s2]);
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) y = mfma2(av[s2], iv[s2], y);
        }
        khalf_reduce(y, red, blk, kh, lane);
        if (kh == 0)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = 8 * (q >> 2) + 4 * lh + (q & 3);
                S[i * SP + jc] = y[q];
                m = fmaxf(m, fabsf(y[q]));
            }
        __syncthreads();
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) iv[s2] = ivn[s2];
    }
    return strip_max(m, red);
}

// Left solve of a 32-column strip S (column j at S + j*SP): Y <- L^-1 S,
// Y_I = Linv_I (S_I - sum_{J<I} L_IJ Y_J).  T: L11 column-major (ld),
// linv: the 64x64 diagonal-block inverses, column-major.  Loads are
// pipelined as in the right solve.
MXP_DEV float strip_left_solve(float* S, int SP, int nbk, const float* __restrict__ T, int ld,
                                  const float* __restrict__ linv, float* red) {
    float m = 0.0f;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 31, lh = lane >> 5, blk = wave & 1, kh = wave >> 1;
    const int k0 = kh * 32 + lh;
    auto ld_iv = [&](float* v, int I) {
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) v[s2] = linv[(int64_t)I * 4096 + (blk * 32 + lr) + 64 * (k0 + 2 * s2)];
    };
    const int ld2 = 2 * ld;
    auto ld_blk = [&](float* av, int J, int I) {
        const float* ub = T + I * 64 + blk * 32 + (int64_t)(J * 64 + kh * 32) * ld;
        const int lo = lr + lh * ld;
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) av[s2] = ub[s2 * ld2 + lo];
    };
    float iv[16], ivn[16], a0[16], a1[16];
    ld_iv(iv, 0);
    for (int I = 0; I < nbk; ++I) {
        f16v_t acc = {};
        auto mf_blk = [&](const float* av, int J) {
            const int kb0 = J * 64 + k0;
            float bv[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) bv[s2] = S[lr * SP + kb0 + 2 * s2];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) pin_f(bv[s2]);
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) acc = mfma2(av[s2], bv[s2], acc);
        };
        // a0 holds block (I, 0) for I > 0 (loaded during step I - 1)
        int J = 0;
        for (; J + 1 < I; J += 2) {
            ld_blk(a1, J + 1, I);
            mf_blk(a0, J);
            if (J + 2 < I) ld_blk(a0, J + 2, I);
            mf_blk(a1, J + 1);
        }
        if (J < I) mf_blk(a0, J);
        if (I + 1 < nbk) {
            ld_blk(a0, 0, I + 1);
            ld_iv(ivn, I + 1);
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
            float bv[16];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) bv[s2] = S[lr * SP + I * 64 + k0 + 2 * s2];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) pin_f(bv[s2]);
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) y = mfma2(iv[s2], bv[s2], y);
        }
        khalf_reduce(y, red, blk, kh, lane);
        if (kh == 0)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = I * 64 + blk * 32 + 8 * (q >> 2) + 4 * lh + (q & 3);
                S[lr * SP + i] = y[q];
                m = fmaxf(m, fabsf(y[q]));
            }
        __syncthreads();
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) iv[s2] = ivn[s2];
    }
    return strip_max(m, red);
}

// LDS of a strip kernel: the strip (32 x (nb+1) floats) and the K-half reduction buffer
static inline size_t trsm_smem(int nb) { return (size_t)(SR * (nb + 1) + 2 * 16 * 64) * sizeof(float); }

// L21 strip: X (32 x nb) = A21[rows, :] U11^-1, then amax -> power-of-two
// scales; writes the operand Lq (K-major, update format, scaled), the stored
// L21 (storage format, scaled) and the scales.  A full strip moves through
// 4-element accesses (a lane: 4 rows of one column of A, 4 columns of one
// row of Lq), with every load of the strip in flight at once; the ragged
// last strip takes element accesses.
template <int ST, int OP>
MXP_DEV void trsm_L_strip(typename Store<ST>::T* A, int64_t lda, int64_t n, int64_t k, int nb,
                          const float* __restrict__ Urm, const float* __restrict__ uinv,
                          typename Operand<OP>::T* Lq, float* inv_sa, float* lsc_blk, float* smem, int w) {
    typedef typename Store<ST>::T STT;
    typedef typename Operand<OP>::T OPT;
    const int SP = nb + 1;
    float* S = smem;
    float* red = smem + SR * SP;
    const int tid = threadIdx.x;
    const int64_t r0 = k + nb + (int64_t)SR * w;
    int64_t rv = n - r0;
    rv = rv > SR ? SR : (rv < 0 ? 0 : rv);
    const bool vec = rv == SR && (r0 & 3) == 0 && (lda & 3) == 0 && ((uintptr_t)A & 15) == 0;
    const int rq = tid & 7, cg = tid >> 3;          // vector mapping: rows 4 rq.., column cg + 32 i
    if (vec) {
        for (int c0 = 0; c0 < nb; c0 += 512) {
            // loads without conditions (a column past nb reads column 0,
            // unused): a load under a branch ends in a wait for every load in
            // flight, which would serialise them
            Pack4<STT> x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int c = c0 + cg + 32 * i;
                x[i] = *(const Pack4<STT>*)(A + (r0 + 4 * rq) + (k + (c < nb ? c : 0)) * lda);
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int c = c0 + cg + 32 * i;
                if (c < nb)
#pragma unroll
                    for (int q = 0; q < 4; ++q) S[(4 * rq + q) * SP + c] = Store<ST>::load(x[i].v, q);
            }
        }
    } else {
        const int ii = tid & 31;
        for (int c = tid >> 5; c < nb; c += 8)
            S[ii * SP + c] = (ii < rv) ? Store<ST>::load(A, (r0 + ii) + (k + c) * lda) : 0.0f;
    }
    __syncthreads();
    const float amax = strip_right_solve(S, SP, nb / 64, Urm, nb, uinv, red);
    const float s_op = Operand<OP>::scaled ? pow2_scale(amax, Operand<OP>::scale_exp) : 1.0f;
    const float s_st = Store<ST>::scaled ? pow2_scale(amax, Store<ST>::scale_exp) : 1.0f;
    if (tid == 0) {
        inv_sa[w] = 1.0f / s_op;
        if (rv > 0) lsc_blk[r0 / SR] = s_st;
    }
    // operand rows (nb contiguous values each): 4 columns per lane
    OPT* Lw = Lq + (int64_t)SR * w * nb;
    for (int e = 4 * tid; e < SR * nb; e += 1024) {
        const int ii = e / nb, c = e - ii * nb;      // nb is a multiple of 64: a lane's 4 stay in one row
        Pack4<OPT> o;
#pragma unroll
        for (int q = 0; q < 4; ++q) o.v[q] = Operand<OP>::from_f32(S[ii * SP + c + q] * s_op);
        *(Pack4<OPT>*)(Lw + e) = o;
    }
    if (vec) {
        for (int c = cg; c < nb; c += 32) {
            Pack4<STT> o;
#pragma unroll
            for (int q = 0; q < 4; ++q) o.v[q] = Store<ST>::from_f32(S[(4 * rq + q) * SP + c] * s_st);
            *(Pack4<STT>*)(A + (r0 + 4 * rq) + (k + c) * lda) = o;
        }
    } else {
        const int ii = tid & 31;
        if (ii < rv)
            for (int c = tid >> 5; c < nb; c += 8) A[(r0 + ii) + (k + c) * lda] = Store<ST>::from_f32(S[ii * SP + c] * s_st);
    }
}

// U12 strip: Y (nb x 32) = L11^-1 A12[:, cols]; operand Uq (K-major: column
// j has nb contiguous values) scaled, stored U12 unscaled.  Accesses as in
// the L21 strip, a lane taking 4 consecutive rows of one column.
template <int ST, int OP>
MXP_DEV void trsm_U_strip(typename Store<ST>::T* A, int64_t lda, int64_t n, int64_t k, int nb,
                          const float* __restrict__ T, const float* __restrict__ linv,
                          typename Operand<OP>::T* Uq, float* inv_sb, float* smem, int w) {
    typedef typename Store<ST>::T STT;
    typedef typename Operand<OP>::T OPT;
    const int SP = nb + 1;
    float* S = smem;
    float* red = smem + SR * SP;
    const int tid = threadIdx.x;
    const int64_t c0 = k + nb + (int64_t)SR * w;
    int64_t cv = n - c0;
    cv = cv > SR ? SR : (cv < 0 ? 0 : cv);
    // nb divides 1024: a pass covers 1024 / nb columns, a lane 4 rows
    const int qpc = nb >> 2, lq = __builtin_ctz((unsigned)qpc);
    const int kq = tid & (qpc - 1), cs = tid >> lq, cpp = 256 >> lq;
    const bool vec = (1024 % nb) == 0 && (k & 3) == 0 && (lda & 3) == 0 && ((uintptr_t)A & 15) == 0;
    if (vec) {
        for (int p0 = 0; p0 < SR; p0 += 16 * cpp) {
            // loads without conditions, as in the L21 strip (a column past the
            // matrix reads column k + nb, unused)
            Pack4<STT> x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int cc = p0 + cs + cpp * i;
                const int64_t col = (cc < SR && cc < cv) ? c0 + cc : k + nb;
                x[i] = *(const Pack4<STT>*)(A + (k + 4 * kq) + col * lda);
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int cc = p0 + cs + cpp * i;
                if (cc < SR)
#pragma unroll
                    for (int q = 0; q < 4; ++q) S[cc * SP + 4 * kq + q] = (cc < cv) ? Store<ST>::load(x[i].v, q) : 0.0f;
            }
        }
    } else {
        for (int cc = 0; cc < SR; ++cc)
            for (int kk = tid; kk < nb; kk += 256)
                S[cc * SP + kk] = (cc < cv) ? Store<ST>::load(A, (k + kk) + (c0 + cc) * lda) : 0.0f;
    }
    __syncthreads();
    const float amax = strip_left_solve(S, SP, nb / 64, T, nb, linv, red);
    const float s_op = Operand<OP>::scaled ? pow2_scale(amax, Operand<OP>::scale_exp) : 1.0f;
    if (tid == 0) inv_sb[w] = 1.0f / s_op;
    OPT* Uw = Uq + (int64_t)SR * w * nb;
    if (vec) {
        for (int cc = cs; cc < SR; cc += cpp) {
            Pack4<OPT> o;
#pragma unroll
            for (int q = 0; q < 4; ++q) o.v[q] = Operand<OP>::from_f32(S[cc * SP + 4 * kq + q] * s_op);
            *(Pack4<OPT>*)(Uw + (int64_t)cc * nb + 4 * kq) = o;
            if (cc < cv) {
                Pack4<STT> a;
#pragma unroll
                for (int q = 0; q < 4; ++q) a.v[q] = Store<ST>::from_f32(S[cc * SP + 4 * kq + q]);
                *(Pack4<STT>*)(A + (k + 4 * kq) + (c0 + cc) * lda) = a;
            }
        }
    } else {
        for (int cc = 0; cc < SR; ++cc)
            for (int kk = tid; kk < nb; kk += 256) {
                Uw[(int64_t)cc * nb + kk] = Operand<OP>::from_f32(S[cc * SP + kk] * s_op);
                if (cc < cv) A[(k + kk) + (c0 + cc) * lda] = Store<ST>::from_f32(S[cc * SP + kk]);
            }
    }
}

// Both strip solves of one block step in one launch: work-groups [0, nstrip)
// solve the L21 strips, [nstrip, 2 nstrip) the U12 strips (independent).  One
// launch serves a group of factorisations (one per request of the solve
// server, or a single one): their work-groups are numbered one after another.
struct TrsmOne {
    void* A;
    int64_t lda, n, k;
    int nb, nstrip, wg_end, pad;
    const float *Urm, *uinv, *T, *linv;
    void* Lq;
    float* inv_sa;
    float* lsc_blk;
    void* Uq;
    float* inv_sb;
};
struct TrsmGroup {
    TrsmOne g[GEMM_GROUP_MAX];
    int count;
};

template <int ST, int OP>
__global__ __launch_bounds__(256) void k_trsm(const TrsmGroup grp) {
    extern __shared__ float smem[];
    int d = 0;
    while ((int)blockIdx.x >= grp.g[d].wg_end) ++d;
    const TrsmOne& G = grp.g[d];
    const int w = (int)blockIdx.x - (d > 0 ? grp.g[d - 1].wg_end : 0);
    typename Store<ST>::T* A = (typename Store<ST>::T*)G.A;
    if (w < G.nstrip)
        trsm_L_strip<ST, OP>(A, G.lda, G.n, G.k, G.nb, G.Urm, G.uinv, (typename Operand<OP>::T*)G.Lq, G.inv_sa,
                             G.lsc_blk, smem, w);
    else
        trsm_U_strip<ST, OP>(A, G.lda, G.n, G.k, G.nb, G.T, G.linv, (typename Operand<OP>::T*)G.Uq, G.inv_sb, smem,
                             w - G.nstrip);
}

// Full FP32 inverses of a diagonal block (size kbp) by strips of 32:
// U11^-1 rows r0..r0+31 = I[r0:r0+32, :] U11^-1 (right solve with Trm, the
// factor row-major), L11^-1 columns c0..c0+31 = L11^-1 I[:, c0:c0+32] (left
// solve with T, column-major); out: the inverse, column-major, ld D.
MXP_DEV void inv_upper_strip(int kbp, const float* __restrict__ Trm, int ld, const float* __restrict__ uinv,
                             float* __restrict__ out, int64_t D, int r0, float* smem) {
    const int SP = kbp + 1;
    float* S = smem;
    float* red = smem + SR * SP;
    for (int e = threadIdx.x; e < SR * kbp; e += 256) {
        int ii = e % SR, c = e / SR;
        S[ii * SP + c] = (r0 + ii == c) ? 1.0f : 0.0f;
    }
    __syncthreads();
    strip_right_solve(S, SP, kbp / 64, Trm, ld, uinv, red);
    for (int e = threadIdx.x; e < SR * kbp; e += 256) {
        int ii = e % SR, c = e / SR;
        out[(r0 + ii) + (int64_t)c * D] = S[ii * SP + c];
    }
}
MXP_DEV void inv_lower_strip(int kbp, const float* __restrict__ T, int ld, const float* __restrict__ linv,
                             float* __restrict__ out, int64_t D, int c0, float* smem) {
    const int SP = kbp + 1;
    float* S = smem;
    float* red = smem + SR * SP;
    for (int e = threadIdx.x; e < SR * kbp; e += 256) {
        int kk = e % kbp, cc = e / kbp;
        S[cc * SP + kk] = (kk == c0 + cc) ? 1.0f : 0.0f;
    }
    __syncthreads();
    strip_left_solve(S, SP, kbp / 64, T, ld, linv, red);
    for (int e = threadIdx.x; e < SR * kbp; e += 256) {
        int kk = e % kbp, cc = e / kbp;
        out[kk + (int64_t)(c0 + cc) * D] = S[cc * SP + kk];
    }
}

// the inverses of diagonal blocks blk0.. in one launch (after the
// factorisation: every block with FP32 storage, the blocks whose strips were
// solved by substitution otherwise); blockIdx.y = block - blk0, blockIdx.x = strip.  Block blk is
// diagonal block blk % g of the preconditioner's group blk / g
// (column-major, ld D).
__global__ __launch_bounds__(256) void k_inv_upper(int64_t n, int nb, int64_t blk0, const float* __restrict__ Trm_all,
                                                   const float* __restrict__ uinv_all, float* __restrict__ out_all) {
    extern __shared__ float smem[];
    const int64_t blk = blk0 + blockIdx.y;
    const int64_t k = blk * nb;
    const int kb = (int)(n - k < nb ? n - k : nb);
    const int kbp = (kb + 63) / 64 * 64;
    const int r0 = SR * blockIdx.x;
    if (r0 >= kbp) return;
    const int64_t D = prec_block(nb), g = D / nb, o = (blk % g) * nb;
    inv_upper_strip(kbp, Trm_all + blk * nb * nb, nb, uinv_all + blk * nb * 64,
                    out_all + (blk / g) * D * D + o + o * D, D, r0, smem);
}

__global__ __launch_bounds__(256) void k_inv_lower(int64_t n, int nb, int64_t blk0, const float* __restrict__ Tall,
                                                   const float* __restrict__ linv_all, float* __restrict__ out_all) {
    extern __shared__ float smem[];
    const int64_t blk = blk0 + blockIdx.y;
    const int64_t k = blk * nb;
    const int kb = (int)(n - k < nb ? n - k : nb);
    const int kbp = (kb + 63) / 64 * 64;
    const int c0 = SR * blockIdx.x;
    if (c0 >= kbp) return;
    const int64_t D = prec_block(nb), g = D / nb, o = (blk % g) * nb;
    inv_lower_strip(kbp, Tall + blk * nb * nb, nb, linv_all + blk * nb * 64,
                    out_all + (blk / g) * D * D + o + o * D, D, c0, smem);
}

// the inverses of one block step's diagonal blocks (16-bit storage: formed
// right after each diagonal-block LU, they serve the strip products and
// later the preconditioner): work-groups [0, kbp/32) of a descriptor solve
// the strips of L11^-1, the next kbp/32 those of U11^-1
__global__ __launch_bounds__(256) void k_block_inv(const PanelGroup grp) {
    extern __shared__ float smem[];
    int d = 0;
    while ((int)blockIdx.x >= grp.g[d].wg_inv) ++d;
    const PanelOne& G = grp.g[d];
    const int w0 = (int)blockIdx.x - (d > 0 ? grp.g[d - 1].wg_inv : 0);
    const int nstr = G.kbp / SR;
    if (w0 < nstr) inv_lower_strip(G.kbp, G.T, G.nb, G.linv, G.Li, G.ldi, SR * w0, smem);
    else inv_upper_strip(G.kbp, G.Trm, G.nb, G.uinv, G.Ui, G.ldi, SR * (w0 - nstr), smem);
}

hipError_t block_inverses(const PanelGroup& grp, int wg, int nbmax, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_block_inv,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)trsm_smem(1024));
    if (attr) return attr;
    k_block_inv<<<wg, 256, trsm_smem(nbmax), s>>>(grp);
    return hipGetLastError();
}

// Off-diagonal blocks of the inverses of the pairs of diagonal blocks
// (blocks b0 = 2p, b1 = 2p + 1 of sizes nb and kb1):
//   [[L0, 0], [B, L1]]^-1 = [[L0^-1, 0], [-L1^-1 B L0^-1, L1^-1]],
//   [[U0, B'], [0, U1]]^-1 = [[U0^-1, -U0^-1 B' U1^-1], [0, U1^-1]],
// with B and B' the stored panels of the factor (B with its strip factors
// undone) and the diagonal inverses from k_inv_lower / k_inv_upper.  Each
// product is one launch over all pairs (blockIdx.z = pair) of 64 x 64
// output tiles on the FP32 matrix cores; the K range of a tile skips the
// zero triangle of its triangular operand.
// LDS pitches of the staged operands (64 banks): A is written with the rows
// running over the lanes and read two k rows at a time (pitch 96: the two
// rows fall on distinct banks); B is written with k running over the lanes
// (pitch 97, odd: 32 consecutive k rows on distinct banks)
constexpr int PP_SP = 96, PP_SPB = 97;

// acc (wave (wr, wc)'s 32 x 32 part of the 64 x 64 tile) += A[i0.., k] B[k, j0..] over k in [k_lo, k_hi);
// the next chunk's operands are loaded into registers before this chunk's
// products, so that their latency overlaps them
template <class FA, class FB>
MXP_DEV f16v_t pair_tile(FA fa, FB fb, int M, int N, int i0, int j0, int k_lo, int k_hi, float* sA, float* sB) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave & 1, wc = wave >> 1, lr = lane & 31, lh = lane >> 5;
    f16v_t acc = {};
    float ra[8], rb[8];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            // loads without conditions (an index past the range reads a
            // valid element, weighted zero): a load under a branch would
            // wait for every load in flight
            const int i = i0 + (e & 63), k = k0 + (e >> 6);          // A: rows contiguous
            const float a = fa(i < M ? i : M - 1, k < k_hi ? k : k_hi - 1);
            ra[t] = (i < M && k < k_hi) ? a : 0.0f;
            const int kq = k0 + (e & 31), j = j0 + (e >> 5);         // B: k contiguous
            const float b = fb(kq < k_hi ? kq : k_hi - 1, j < N ? j : N - 1);
            rb[t] = (j < N && kq < k_hi) ? b : 0.0f;
        }
    };
    if (k_lo < k_hi) fetch(k_lo);
    for (int k0 = k_lo; k0 < k_hi; k0 += 32) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = tid + 256 * t;
            sA[(e >> 6) * PP_SP + (e & 63)] = ra[t];
            sB[(e & 31) * PP_SPB + (e >> 5)] = rb[t];
        }
        __syncthreads();
        if (k0 + 32 < k_hi) fetch(k0 + 32);
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) {
            const int kk = 2 * s2 + lh;
            acc = mfma2(sA[kk * PP_SP + wr * 32 + lr], sB[kk * PP_SPB + wc * 32 + lr], acc);
        }
        __syncthreads();
    }
    return acc;
}

// C[i][j] = alpha acc, register q of lane l holding row 8(q/4) + 4(l/32) + q%4, column l%32
template <class FC>
MXP_DEV void pair_store(const f16v_t& acc, float alpha, int M, int N, int i0, int j0, FC fc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave & 1, wc = wave >> 1;
    const int j = j0 + wc * 32 + (lane & 31);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = i0 + wr * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        if (i < M && j < N) fc(i, j, alpha * acc[q]);
    }
}

// phase 0: W = B L0^-1 (kb1 x nb, ld nb, into W), phase 1: X = -L1^-1 W
template <int ST>
__global__ __launch_bounds__(256) void k_pair_lower(int64_t n, int nb, const typename Store<ST>::T* __restrict__ A,
                                                    int64_t lda, const float* __restrict__ lsc, int64_t nstrips32,
                                                    float* __restrict__ inv_all, float* __restrict__ W, int phase) {
    __shared__ float sA[32 * PP_SP], sB[32 * PP_SPB];
    const int64_t p = blockIdx.z, D = 2 * (int64_t)nb;
    const int64_t k0 = p * D, k1 = k0 + nb;
    if (k1 >= n) return;
    const int kb1 = (int)(n - k1 < nb ? n - k1 : nb);
    float* inv = inv_all + p * D * D;
    float* Wp = W + p * (int64_t)nb * nb;
    const int i0 = 64 * blockIdx.y, j0 = 64 * blockIdx.x;
    if (phase == 0) {
        if (i0 >= kb1) return;
        const float* srow = lsc + (2 * p) * nstrips32;
        auto fa = [&](int i, int k) {
            return Store<ST>::load(A, (k1 + i) + (k0 + k) * lda) / srow[(k1 + i) / 32];
        };
        auto fb = [&](int k, int j) { return inv[k + (int64_t)j * D]; };
        const f16v_t acc = pair_tile(fa, fb, kb1, nb, i0, j0, j0, nb, sA, sB);   // L0^-1[k][j] = 0 for k < j
        pair_store(acc, 1.0f, kb1, nb, i0, j0, [&](int i, int j, float v) { Wp[i + (int64_t)j * nb] = v; });
    } else {
        if (i0 >= kb1) return;
        auto fa = [&](int i, int k) { return inv[(nb + i) + (int64_t)(nb + k) * D]; };
        auto fb = [&](int k, int j) { return Wp[k + (int64_t)j * nb]; };
        const int kh = i0 + 64 < kb1 ? i0 + 64 : kb1;                             // L1^-1[i][k] = 0 for k > i
        const f16v_t acc = pair_tile(fa, fb, kb1, nb, i0, j0, 0, kh, sA, sB);
        pair_store(acc, -1.0f, kb1, nb, i0, j0, [&](int i, int j, float v) { inv[(nb + i) + (int64_t)j * D] = v; });
    }
}

// phase 0: W = U0^-1 B' (nb x kb1, ld nb, into W), phase 1: Y = -W U1^-1
template <int ST>
__global__ __launch_bounds__(256) void k_pair_upper(int64_t n, int nb, const typename Store<ST>::T* __restrict__ A,
                                                    int64_t lda, float* __restrict__ inv_all, float* __restrict__ W,
                                                    int phase) {
    __shared__ float sA[32 * PP_SP], sB[32 * PP_SPB];
    const int64_t p = blockIdx.z, D = 2 * (int64_t)nb;
    const int64_t k0 = p * D, k1 = k0 + nb;
    if (k1 >= n) return;
    const int kb1 = (int)(n - k1 < nb ? n - k1 : nb);
    float* inv = inv_all + p * D * D;
    float* Wp = W + p * (int64_t)nb * nb;
    const int i0 = 64 * blockIdx.y, j0 = 64 * blockIdx.x;
    if (j0 >= kb1) return;
    if (phase == 0) {
        auto fa = [&](int i, int k) { return inv[i + (int64_t)k * D]; };
        auto fb = [&](int k, int j) { return Store<ST>::load(A, (k0 + k) + (k1 + j) * lda); };
        const f16v_t acc = pair_tile(fa, fb, nb, kb1, i0, j0, i0, nb, sA, sB);   // U0^-1[i][k] = 0 for k < i
        pair_store(acc, 1.0f, nb, kb1, i0, j0, [&](int i, int j, float v) { Wp[i + (int64_t)j * nb] = v; });
    } else {
        auto fa = [&](int i, int k) { return Wp[i + (int64_t)k * nb]; };
        auto fb = [&](int k, int j) { return inv[(nb + k) + (int64_t)(nb + j) * D]; };
        const int kh = j0 + 64 < kb1 ? j0 + 64 : kb1;                             // U1^-1[k][j] = 0 for k > j
        const f16v_t acc = pair_tile(fa, fb, nb, kb1, i0, j0, 0, kh, sA, sB);
        pair_store(acc, -1.0f, nb, kb1, i0, j0, [&](int i, int j, float v) { inv[i + (int64_t)(nb + j) * D] = v; });
    }
}

// the full FP32 inverses of the preconditioner's diagonal blocks (after the
// factorisation): every factor block's, then the off-diagonal blocks of the
// pairs.  W: scratch of ceil(n / 2nb) nb^2 floats.
// Block step k solves its strips through the block inverses (16-bit storage)
// while the trailing part is at least MXP_PANEL_MIN blocks: there the
// products free the compute units the substitution would hold beside the
// merged update; the last steps, bound by the chain of panel solves, keep the
// substitution, whose latency is lower.  Depends on (n, nb, k) alone, so that
// grouped and single factorisations take the same path.
#ifndef MXP_PANEL_MIN
#define MXP_PANEL_MIN 16
#endif
static bool inverse_path(const FactorPlan& p, int64_t k) {
    const int64_t kb = p.n - k < p.nb ? p.n - k : p.nb;
    return panel_path(p.store) && p.n - k - kb >= MXP_PANEL_MIN * p.nb;
}
// the first block whose inverses are formed after the factorisation
static int64_t inv_first_after(const FactorPlan& p) {
    const int64_t nblk = (p.n + p.nb - 1) / p.nb;
    int64_t b = 0;
    while (b < nblk && inverse_path(p, b * p.nb)) ++b;
    return b;
}

template <int ST>
static hipError_t prec_inverses(const FactorPlan& p, float* W, hipStream_t s) {
    const int64_t n = p.n, nb = p.nb;
    const int64_t nblk = (n + nb - 1) / nb;
    // blocks before blk0 got their inverses during the factorisation
    const int64_t blk0 = inv_first_after(p);
    dim3 g((unsigned)(nb / SR), (unsigned)(nblk - blk0));
    hipEvent_t pt = prof::begin(prof::DIAG, s);
    if (blk0 < nblk) {
        k_inv_upper<<<g, 256, trsm_smem((int)nb), s>>>(n, (int)nb, blk0, p.Trm, p.uinv, p.uinv_full);
        k_inv_lower<<<g, 256, trsm_smem((int)nb), s>>>(n, (int)nb, blk0, p.T, p.linv, p.linv_full);
    }
    double fl = 2.0 / 3.0 * (double)n * nb * nb;
    if (prec_block(nb) == 2 * nb && n > nb) {
        const int64_t npair = (n + 2 * nb - 1) / (2 * nb);
        const dim3 gp((unsigned)(nb / 64), (unsigned)(nb / 64), (unsigned)npair);
        typedef typename Store<ST>::T T;
        // the lower and then the upper products, each pair of launches through W
        for (int ph = 0; ph < 2; ++ph)
            k_pair_lower<ST><<<gp, 256, 0, s>>>(n, (int)nb, (const T*)p.A, p.lda, p.lsc, (n + 31) / 32, p.linv_full,
                                                W, ph);
        for (int ph = 0; ph < 2; ++ph)
            k_pair_upper<ST><<<gp, 256, 0, s>>>(n, (int)nb, (const T*)p.A, p.lda, p.uinv_full, W, ph);
        fl += 4.0 * (double)n * nb * nb;
    }
    prof::end(pt, prof::DIAG, s, fl, 16.0 * (double)n * nb);
    return hipGetLastError();
}

// ============================================================== driver

hipError_t lookahead_create(Lookahead* la) {
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&la->side, hipStreamNonBlocking))) return e;
    if ((e = hipEventCreateWithFlags(&la->ev_upd, hipEventDisableTiming))) return e;
    if ((e = hipEventCreateWithFlags(&la->ev_cross, hipEventDisableTiming))) return e;
    if ((e = hipEventCreateWithFlags(&la->ev_next, hipEventDisableTiming))) return e;
    return hipEventCreateWithFlags(&la->ev_panel, hipEventDisableTiming);
}

void lookahead_destroy(Lookahead* la) {
    if (la->ev_panel) (void)hipEventDestroy(la->ev_panel);
    if (la->ev_next) (void)hipEventDestroy(la->ev_next);
    if (la->ev_cross) (void)hipEventDestroy(la->ev_cross);
    if (la->ev_upd) (void)hipEventDestroy(la->ev_upd);
    if (la->side) (void)hipStreamDestroy(la->side);
    *la = Lookahead();
}

// Look-ahead contexts of callers that bring none: a pool per device
// (default stream priority).  A call takes a context for the time it
// enqueues its work and returns it afterwards; work still in flight on the
// context's side stream is no hazard for the next user, whose waits and
// records are enqueued after it (a wait on an event refers to the event's
// latest record at the time of the wait call).  Two calls never enqueue on
// one context at the same time.
static std::vector<Lookahead*> g_la_free[64];
static std::mutex g_la_mutex;

static hipError_t lookahead_acquire(int dev, Lookahead** out) {
    {
        std::lock_guard<std::mutex> lock(g_la_mutex);
        if (!g_la_free[dev].empty()) {
            *out = g_la_free[dev].back();
            g_la_free[dev].pop_back();
            return hipSuccess;
        }
    }
    Lookahead* L = new Lookahead();
    hipError_t e = lookahead_create(L);
    if (e) {
        lookahead_destroy(L);
        delete L;
        return e;
    }
    *out = L;
    return hipSuccess;
}

static void lookahead_release(int dev, Lookahead* L) {
    std::lock_guard<std::mutex> lock(g_la_mutex);
    g_la_free[dev].push_back(L);
}

// the strip-TRSM descriptor of block step k of a factorisation; wg_begin: the
// work-groups of the group before it
template <int ST, int OP>
static void trsm_desc(const FactorPlan& p, int64_t k, TrsmOne& g, int wg_begin) {
    typedef typename Operand<OP>::T OP_T;
    const int nb = (int)p.nb;
    const int kb = (int)(p.n - k < nb ? p.n - k : nb);
    const int64_t m = p.n - k - kb;
    const int64_t blk = k / nb;
    const int set = (int)(blk & 3);
    const int64_t opset = p.op_rows * nb, scset = p.op_rows / 32;
    const int nstrip = (int)(rup(m, 256) / SR);
    g.A = p.A; g.lda = p.lda; g.n = p.n; g.k = k; g.nb = nb; g.nstrip = nstrip;
    g.wg_end = wg_begin + 2 * nstrip;
    g.pad = 0;
    g.Urm = p.Trm + blk * nb * nb;
    g.uinv = p.uinv + blk * nb * 64;
    g.T = p.T + blk * nb * nb;
    g.linv = p.linv + blk * nb * 64;
    g.Lq = (OP_T*)p.Lq + set * opset;
    g.inv_sa = p.inv_sa + set * scset;
    g.lsc_blk = p.lsc + blk * ((p.n + SR - 1) / SR);
    g.Uq = (OP_T*)p.Uq + set * opset;
    g.inv_sb = p.inv_sb + set * scset;
}

// The descriptor of block step k for the inverse-based strip solves; tr:
// the output tile rows of the panel_trsm launch (panel_rows of the largest
// nb it serves); wg0: the first work-group numbers of the three launches.
// Blocks without a trailing part (the last) only get their inverses.
static void panel_desc(const FactorPlan& p, int64_t k, int tr, PanelOne& g, const int wg0[3]) {
    const int nb = (int)p.nb;
    const int kb = (int)(p.n - k < nb ? p.n - k : nb);
    const int64_t m = p.n - k - kb;
    const int64_t blk = k / nb;
    const int set = (int)(blk & 3);
    const int eb = dtype_bytes(p.update);
    const int64_t opset = p.op_rows * nb, scset = p.op_rows / 32;
    const int64_t D = prec_block(nb), gsz = D / nb, o = (blk % gsz) * nb;
    g.A = p.A; g.lda = p.lda; g.n = p.n; g.k = k; g.ldi = D;
    g.nb = nb; g.kbp = (int)rup(kb, 64);
    g.ntile = m > 0 ? (int)(rup(m, 256) / tr) : 0;
    g.pad = g.pad2 = 0;
    g.wg_inv = wg0[0] + 2 * (g.kbp / SR);
    g.wg_split = wg0[1] + (m > 0 ? 2 * (nb / 16) : 0);
    g.wg_trsm = wg0[2] + 2 * g.ntile;
    g.T = p.T + blk * nb * nb;
    g.Trm = p.Trm + blk * nb * nb;
    g.linv = p.linv + blk * nb * 64;
    g.uinv = p.uinv + blk * nb * 64;
    g.Li = p.linv_full + (blk / gsz) * D * D + o + o * D;
    g.Ui = p.uinv_full + (blk / gsz) * D * D + o + o * D;
    g.ub = p.binv;
    g.lb = (char*)p.binv + (size_t)3 * nb * nb * 2;
    g.ubs = p.binv_sc;
    g.lbs = p.binv_sc + nb;
    g.Lq = (char*)p.Lq + (size_t)set * opset * eb;
    g.inv_sa = p.inv_sa + set * scset;
    g.lsc_blk = p.lsc + blk * ((p.n + SR - 1) / SR);
    g.Uq = (char*)p.Uq + (size_t)set * opset * eb;
    g.inv_sb = p.inv_sb + set * scset;
}

// The trailing updates of the block steps, taken in pairs: block column and
// row k+1 receive the update of step k alone (they form panel k+1), and
// everything beyond them the updates of steps k and k+1 in one pass with K =
// 2 nb (one rounding to the storage format instead of two, half the C
// traffic).  With steps (k, k+1) a pair (k even in blocks), every element is
// computed by the same arithmetic however the updates are cut into launches.
//
// The operands of step j sit in set (j / nb) & 3 (four sets: two pairs in
// flight); row r of a set belongs to global row (column) j + nb + r.
template <int ST, int OP>
static GemmCall pair_call(const FactorPlan& p, int64_t j, bool pair, int64_t r0, int64_t c0, int64_t M,
                          int64_t N) {
    typedef typename Store<ST>::T ST_T;
    typedef typename Operand<OP>::T OP_T;
    const int64_t nb = p.nb;
    const int64_t opset = p.op_rows * nb, scset = p.op_rows / 32;
    GemmCall g{};
    g.C = (ST_T*)p.A + r0 + c0 * p.lda;
    g.ldc = p.lda;
    g.M = M;
    g.N = N;
    auto seg = [&](int64_t step, const void*& a, const void*& b, const float*& sa, const float*& sb) {
        const int set = (int)((step / nb) & 3);
        const int64_t ro = r0 - step - nb, co = c0 - step - nb;
        a = (const OP_T*)p.Lq + set * opset + ro * nb;
        b = (const OP_T*)p.Uq + set * opset + co * nb;
        sa = p.inv_sa + set * scset + ro / 32;
        sb = p.inv_sb + set * scset + co / 32;
    };
    g.K = (int)nb;
    seg(j, g.Aq, g.Bq, g.inv_sa, g.inv_sb);
    if (pair) {
        g.K2 = (int)nb;
        seg(j + nb, g.Aq2, g.Bq2, g.inv_sa2, g.inv_sb2);
    }
    return g;
}

// the update of block column and row b (width w, from global index b) by
// step j alone or by the pair (j, j+nb): two descriptors
template <int ST, int OP>
static int cross_calls(const FactorPlan& p, int64_t j, bool pair, int64_t b, GemmCall* out) {
    const int64_t n = p.n, w = n - b < p.nb ? n - b : p.nb;
    int c = 0;
    out[c++] = pair_call<ST, OP>(p, j, pair, b, b, n - b, w);               // block column b, diagonal included
    if (n - b - w > 0) out[c++] = pair_call<ST, OP>(p, j, pair, b, b + w, w, n - b - w);   // rest of block row b
    return c;
}

// Right-looking blocked LU with look-ahead, the updates taken in pairs (see
// above).  With the pair (k, k1), k1 = k + nb, and k2, k3 the next two
// blocks, the caller's stream runs the pair's update in two launches -- the
// rest of block column and row k2 (the diagonal block k2 is updated on the
// side stream) with block column and row k3, then everything beyond -- while
// the side stream runs the chain that sets the pace of the late steps: the
// diagonal block k2, its LU, the strip TRSMs of step k2 and the update of
// block column and row k3 by step k2 alone (after the first launch), the LU
// and TRSMs of block k3.  One event per hand-over; in the late steps each
// has fired before its wait is reached.  The operand sets of the pair are
// rewritten by the TRSMs two pairs later, which the side stream enqueues
// after it has seen the pair's last update end.
template <int ST, int OP>
static hipError_t factor_typed(const FactorPlan& p, hipStream_t s, Lookahead* la) {
    typedef typename Store<ST>::T ST_T;
    typedef typename Operand<OP>::T OP_T;
    static const hipError_t attr = []() {
        hipError_t e2;
        if ((e2 = hipFuncSetAttribute((const void*)k_trsm<ST, OP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)trsm_smem(1024)))) return e2;
        if ((e2 = hipFuncSetAttribute((const void*)k_inv_upper, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)trsm_smem(1024)))) return e2;
        return hipFuncSetAttribute((const void*)k_inv_lower, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)trsm_smem(1024));
    }();
    if (attr) return attr;
    hipError_t e;
    Lookahead* LA = la;
    ST_T* A = (ST_T*)p.A;
    constexpr bool NP = ST == F16 || ST == BF16;     // strip solves through the block inverses
    const int64_t n = p.n, lda = p.lda;
    const int nb = (int)p.nb;

    // diagonal-block LU of block k (latency-bound: a handful of small grids)
    auto diag = [&](int64_t k, hipStream_t st) -> hipError_t {
        const int kb = (int)(n - k < nb ? n - k : nb);
        const int kbp = (int)rup(kb, 64);
        const int64_t blk = k / nb;
        float* T = p.T + blk * nb * nb;
        float* linv = p.linv + blk * nb * 64;
        float* uinv = p.uinv + blk * nb * 64;
        hipEvent_t pt = prof::begin(prof::DIAG, st);
        hipError_t e2 = diag_lu(ST, A, lda, k, kb, kbp, T, p.Trm + blk * nb * nb, nb, linv, uinv,
                                p.dsync + blk * diag_sync_words(), p.info, st);
        if (e2) return e2;
        prof::end(pt, prof::DIAG, st, 2.0 / 3.0 * kb * (double)kb * kb, 2.0 * kb * (double)kb * sizeof(ST_T));
        if ((e2 = hipGetLastError())) return e2;
        if (NP && inverse_path(p, k)) {
            // the block's inverses and their 16-bit parts (the strip products' B operands)
            PanelGroup pg;
            const int wg0[3] = {0, 0, 0};
            panel_desc(p, k, panel_rows(ST, nb), pg.g[0], wg0);
            pg.count = 1;
            hipEvent_t pi = prof::begin(prof::TRSM, st);
            if ((e2 = block_inverses(pg, pg.g[0].wg_inv, nb, st))) return e2;
            if (pg.g[0].wg_split > 0 && (e2 = panel_split(ST, pg, pg.g[0].wg_split, nb, st))) return e2;
            prof::end(pi, prof::TRSM, st, 4.0 / 3.0 * kb * (double)kb * kb, 8.0 * kb * (double)kb);
        }
        return hipSuccess;
    };
    // strip TRSMs of block k (wide grids: all CUs)
    auto trsm = [&](int64_t k, hipStream_t st) -> hipError_t {
        const int kb = (int)(n - k < nb ? n - k : nb);
        const int64_t m = n - k - kb;
        if (m <= 0) return hipSuccess;
        if (NP && inverse_path(p, k)) {
            PanelGroup pg;
            const int wg0[3] = {0, 0, 0};
            panel_desc(p, k, panel_rows(ST, nb), pg.g[0], wg0);
            pg.count = 1;
            hipEvent_t pt = prof::begin(prof::TRSM, st);
            hipError_t e2 = panel_trsm(ST, OP, pg, pg.g[0].wg_trsm, nb, st);
            prof::end(pt, prof::TRSM, st, 4.0 * m * (double)nb * nb,
                      4.0 * m * (double)nb * sizeof(ST_T) + 2.0 * m * (double)nb * sizeof(OP_T));
            return e2;
        }
        TrsmGroup grp;
        trsm_desc<ST, OP>(p, k, grp.g[0], 0);
        grp.count = 1;
        hipEvent_t pt = prof::begin(prof::TRSM, st);
        k_trsm<ST, OP><<<grp.g[0].wg_end, 256, trsm_smem(nb), st>>>(grp);
        prof::end(pt, prof::TRSM, st, 2.0 * m * (double)nb * nb,
                  4.0 * m * (double)nb * sizeof(ST_T) + 2.0 * m * (double)nb * sizeof(OP_T));
        return hipGetLastError();
    };
    // one trailing-update launch of up to two descriptors, timed on its own
    auto gemm = [&](const GemmCall* c, int cnt, hipStream_t st) -> hipError_t {
        double fl = 0, by = 0;
        for (int i = 0; i < cnt; ++i) {
            const double K = c[i].K + c[i].K2;
            fl += 2.0 * c[i].M * (double)c[i].N * K;
            by += 2.0 * c[i].M * (double)c[i].N * sizeof(ST_T) + (c[i].M + c[i].N) * K * sizeof(OP_T);
        }
        if (fl == 0) return hipSuccess;
        // launches of fewer 256-row tiles than CUs (the late steps, the
        // diagonal block) take 128-row tiles: twice the work-groups, the
        // same arithmetic per element
        int tile = p.gemm_tile;
        int64_t tiles = 0;
        for (int i = 0; i < cnt; ++i) tiles += ((c[i].M + 255) / 256) * ((c[i].N + 127) / 128);
        if (tiles < 256) tile = GEMM_TILE_128;
        hipEvent_t pt = prof::begin(prof::GEMM, st);
        hipError_t e2 = gemm_group(OP, ST, tile, c, cnt, st);
        prof::end(pt, prof::GEMM, st, fl, by);
        return e2;
    };
    // block column and row b by step j (pair: by steps j and j + nb)
    auto cross = [&](int64_t j, bool pair, int64_t b, hipStream_t st) -> hipError_t {
        GemmCall c[2];
        const int cnt = cross_calls<ST, OP>(p, j, pair, b, c);
        return gemm(c, cnt, st);
    };
    // the square [b, n) x [b, n) by the pair (j, j + nb)
    auto square = [&](int64_t j, int64_t b, int64_t w, hipStream_t st) -> hipError_t {
        GemmCall c = pair_call<ST, OP>(p, j, true, b, b, w, w);
        return gemm(&c, 1, st);
    };

    if ((e = fill_u64(p.info, 1, ~0ull, s))) return e;
    {
        const int64_t words = ((n + nb - 1) / nb) * (int64_t)diag_sync_words();
        if ((e = fill_u64(p.dsync, (words + 1) / 2, 0ull, s))) return e;
    }
    // panels 0 and 1 (block column and row 1 updated by step 0 alone)
    if ((e = diag(0, s))) return e;
    if ((e = trsm(0, s))) return e;
    if (nb < n) {
        if ((e = cross(0, false, nb, s))) return e;
        if ((e = diag(nb, s))) return e;
        if ((e = trsm(nb, s))) return e;
    }
    if ((e = hipEventRecord(LA->ev_upd, s))) return e;
    bool side_used = false;
    for (int64_t k = 0; k + 2 * nb < n; k += 2 * nb) {
        // panels k and k1 = k + nb are formed; the pair (k, k1) updates [k2, n)
        const int64_t k2 = k + 2 * nb, k3 = k2 + nb;
        const int64_t w2 = n - k2 < nb ? n - k2 : nb;
        // side: diagonal block k2 (needs the previous pair's last update), its LU
        if ((e = hipStreamWaitEvent(LA->side, LA->ev_upd, 0))) return e;
        if ((e = square(k, k2, w2, LA->side))) return e;
        if ((e = diag(k2, LA->side))) return e;
        // main: the rest of block column and row k2 (needs panel k1) and
        // block column and row k3, in one launch (the side stream's diagonal
        // LU of k2 outlasts both), then everything beyond
        if (side_used && (e = hipStreamWaitEvent(s, LA->ev_panel, 0))) return e;
        {
            GemmCall c[4];
            int cnt = 0;
            if (n - k2 - w2 > 0) {
                c[cnt++] = pair_call<ST, OP>(p, k, true, k2 + w2, k2, n - k2 - w2, w2);
                c[cnt++] = pair_call<ST, OP>(p, k, true, k2, k2 + w2, w2, n - k2 - w2);
            }
            if (k3 < n) cnt += cross_calls<ST, OP>(p, k, true, k3, c + cnt);
            if (cnt && (e = gemm(c, cnt, s))) return e;
        }
        if ((e = hipEventRecord(LA->ev_cross, s))) return e;
        if (k3 < n) {
            const int64_t w3 = n - k3 < nb ? n - k3 : nb;
            if ((e = hipEventRecord(LA->ev_next, s))) return e;
            if (n - k3 - w3 > 0) {
                GemmCall c = pair_call<ST, OP>(p, k, true, k3 + w3, k3 + w3, n - k3 - w3, n - k3 - w3);
                if ((e = gemm(&c, 1, s))) return e;
            }
            if ((e = hipEventRecord(LA->ev_upd, s))) return e;
            // side: panel k2, block column and row k3 by step k2, panel k3
            if ((e = hipStreamWaitEvent(LA->side, LA->ev_cross, 0))) return e;
            if ((e = trsm(k2, LA->side))) return e;
            if ((e = hipStreamWaitEvent(LA->side, LA->ev_next, 0))) return e;
            if ((e = cross(k2, false, k3, LA->side))) return e;
            if ((e = diag(k3, LA->side))) return e;
            if ((e = trsm(k3, LA->side))) return e;
        }
        if ((e = hipEventRecord(LA->ev_panel, LA->side))) return e;
        side_used = true;
    }
    // the caller's stream ends after every side-stream kernel
    if (side_used && (e = hipStreamWaitEvent(s, LA->ev_panel, 0))) return e;
    // full FP32 inverses of the preconditioner's diagonal blocks
    return prec_inverses<ST>(p, p.pairw, s);
}

static hipError_t factor_dispatch(const FactorPlan& p, hipStream_t s, Lookahead* la) {
    const int u = p.update, t = p.store;
    if (u == F32 && t == F32) return factor_typed<F32, F32>(p, s, la);
    if (u == F16 && t == F16) return factor_typed<F16, F16>(p, s, la);
    if (u == BF16 && t == BF16) return factor_typed<BF16, BF16>(p, s, la);
    if (u == F8 && t == F16) return factor_typed<F16, F8>(p, s, la);
    if (u == F8 && t == BF16) return factor_typed<BF16, F8>(p, s, la);
    if (u == F16 && t == F32) return factor_typed<F32, F16>(p, s, la);
    if (u == BF16 && t == F32) return factor_typed<F32, BF16>(p, s, la);
    return hipErrorInvalidValue;
}

template <int ST, int OP>
static hipError_t factor_group_typed(const FactorPlan* P, int count, hipStream_t s) {
    typedef typename Store<ST>::T ST_T;
    typedef typename Operand<OP>::T OP_T;
    constexpr bool NP = ST == F16 || ST == BF16;     // strip solves through the block inverses
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_trsm<ST, OP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)trsm_smem(1024))))
        return e;
    if ((e = hipFuncSetAttribute((const void*)k_inv_upper, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)trsm_smem(1024))))
        return e;
    if ((e = hipFuncSetAttribute((const void*)k_inv_lower, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)trsm_smem(1024))))
        return e;
    int64_t steps = 0;
    for (int g = 0; g < count; ++g) {
        const FactorPlan& p = P[g];
        if ((e = fill_u64(p.info, 1, ~0ull, s))) return e;
        const int64_t nblk = (p.n + p.nb - 1) / p.nb;
        const int64_t words = nblk * (int64_t)diag_sync_words();
        if ((e = fill_u64(p.dsync, (words + 1) / 2, 0ull, s))) return e;
        steps = nblk > steps ? nblk : steps;
    }
    // panel t (diagonal-block LU, strip TRSMs) of every factorisation that has block t
    auto panels = [&](int64_t t) -> hipError_t {
        DiagCall dc[GEMM_GROUP_MAX];
        TrsmGroup tg;
        PanelGroup pg;
        int nd = 0, nt = 0, np = 0, wg = 0, nbmax = 64, pnbmax = 64;
        for (int g = 0; g < count; ++g) {
            const FactorPlan& p = P[g];
            const int nb = (int)p.nb;
            const int64_t k = t * nb;
            if (k >= p.n) continue;
            const int kb = (int)(p.n - k < nb ? p.n - k : nb);
            const int64_t blk = k / nb, m = p.n - k - kb;
            dc[nd++] = DiagCall{p.A, p.lda, k, kb, (int)rup(kb, 64), nb, p.T + blk * nb * nb, p.Trm + blk * nb * nb,
                                p.linv + blk * nb * 64, p.uinv + blk * nb * 64, p.dsync + blk * diag_sync_words(),
                                p.info};
            if (NP && inverse_path(p, k)) {
                pg.g[np++].nb = nb;                       // descriptors filled below (tile rows need nbmax)
                pnbmax = nb > pnbmax ? nb : pnbmax;
                continue;
            }
            if (m <= 0) continue;
            trsm_desc<ST, OP>(p, k, tg.g[nt], wg);
            wg = tg.g[nt++].wg_end;
            nbmax = nb > nbmax ? nb : nbmax;
        }
        if (!nd) return hipSuccess;
        hipError_t e2 = diag_lu_group(ST, dc, nd, s);
        if (e2) return e2;
        if (np) {
            // the steps on the inverse path: inverses, their parts, the strip products
            int wg0[3] = {0, 0, 0}, i = 0;
            for (int g = 0; g < count; ++g) {
                const FactorPlan& p = P[g];
                const int64_t k = t * p.nb;
                if (k >= p.n || !inverse_path(p, k)) continue;
                panel_desc(p, k, panel_rows(ST, pnbmax), pg.g[i], wg0);
                wg0[0] = pg.g[i].wg_inv; wg0[1] = pg.g[i].wg_split; wg0[2] = pg.g[i].wg_trsm;
                ++i;
            }
            pg.count = np;
            hipEvent_t pt = prof::begin(prof::TRSM, s);
            if ((e2 = block_inverses(pg, wg0[0], pnbmax, s))) return e2;
            if ((e2 = panel_split(ST, pg, wg0[1], pnbmax, s))) return e2;
            if ((e2 = panel_trsm(ST, OP, pg, wg0[2], pnbmax, s))) return e2;
            prof::end(pt, prof::TRSM, s, 0.0, 0.0);
        }
        if (!nt) return hipSuccess;
        tg.count = nt;
        hipEvent_t pt = prof::begin(prof::TRSM, s);
        k_trsm<ST, OP><<<wg, 256, trsm_smem(nbmax), s>>>(tg);
        prof::end(pt, prof::TRSM, s, 0.0, 0.0);
        return hipGetLastError();
    };
    auto gemms = [&](const GemmCall* gc, int ng) -> hipError_t {
        if (!ng) return hipSuccess;
        double fl = 0, by = 0;
        for (int i = 0; i < ng; ++i) {
            const double K = gc[i].K + gc[i].K2;
            fl += 2.0 * gc[i].M * (double)gc[i].N * K;
            by += 2.0 * gc[i].M * (double)gc[i].N * sizeof(ST_T) + (gc[i].M + gc[i].N) * K * sizeof(OP_T);
        }
        hipEvent_t pg = prof::begin(prof::GEMM, s);
        hipError_t e2 = gemm_group(OP, ST, P[0].gemm_tile, gc, ng, s);
        prof::end(pg, prof::GEMM, s, fl, by);
        return e2;
    };
    // the updates in pairs of steps, with the arithmetic of mxp_factor:
    // panel t, block column and row t+1 by step t alone, panel t+1, the rest
    // by steps t and t+1 in one pass
    for (int64_t t = 0; t < steps; t += 2) {
        if ((e = panels(t))) return e;
        GemmCall gc[GEMM_DESC_MAX];
        int ng = 0;
        for (int g = 0; g < count; ++g) {
            const FactorPlan& p = P[g];
            const int64_t b = (t + 1) * p.nb;
            if (b < p.n) ng += cross_calls<ST, OP>(p, t * p.nb, false, b, gc + ng);
        }
        if ((e = gemms(gc, ng))) return e;
        if ((e = panels(t + 1))) return e;
        ng = 0;
        for (int g = 0; g < count; ++g) {
            const FactorPlan& p = P[g];
            const int64_t b = (t + 2) * p.nb;
            if (b < p.n) gc[ng++] = pair_call<ST, OP>(p, t * p.nb, true, b, b, p.n - b, p.n - b);
        }
        if ((e = gemms(gc, ng))) return e;
    }
    for (int g = 0; g < count; ++g)
        if ((e = prec_inverses<ST>(P[g], P[g].pairw, s))) return e;
    return hipSuccess;
}

hipError_t factor_group(const FactorPlan* P, int count, hipStream_t s) {
    if (count < 1 || count > GEMM_GROUP_MAX) return hipErrorInvalidValue;
    for (int g = 1; g < count; ++g)
        if (P[g].update != P[0].update || P[g].store != P[0].store) return hipErrorInvalidValue;
    const int u = P[0].update, t = P[0].store;
    if (u == F32 && t == F32) return factor_group_typed<F32, F32>(P, count, s);
    if (u == F16 && t == F16) return factor_group_typed<F16, F16>(P, count, s);
    if (u == BF16 && t == BF16) return factor_group_typed<BF16, BF16>(P, count, s);
    if (u == F8 && t == F16) return factor_group_typed<F16, F8>(P, count, s);
    if (u == F8 && t == BF16) return factor_group_typed<BF16, F8>(P, count, s);
    if (u == F16 && t == F32) return factor_group_typed<F32, F16>(P, count, s);
    if (u == BF16 && t == F32) return factor_group_typed<F32, BF16>(P, count, s);
    return hipErrorInvalidValue;
}

hipError_t factor_run(const FactorPlan& p, hipStream_t s, Lookahead* la) {
    if (la) return factor_dispatch(p, s, la);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    Lookahead* L = nullptr;
    if ((e = lookahead_acquire(dev, &L))) return e;
    e = factor_dispatch(p, s, L);
    lookahead_release(dev, L);
    return e;
}

}  // namespace mxp
