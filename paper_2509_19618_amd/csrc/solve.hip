// solve.hip -- FP64 pieces of the GMRES-based refinement (paper:
// "Algorithmic Framework": the low-precision factors used as a left
// preconditioner, GMRES in 64-bit, at most 50 iterations).
//
// prec_apply: z = U^-1 L^-1 S v by block forward and backward substitution
// on the stored factor (FP64 arithmetic): the nb x nb diagonal blocks use the
// FP32 L11\U11 kept by the factorisation with the inverses of their 64x64
// diagonal sub-blocks; the off-diagonal panels are read in the storage
// format (L21 strips unscaled by their power-of-two factor).
// Modified Gram-Schmidt, Givens rotations, the least-squares solve and the
// basis update are deterministic (fixed reduction orders).
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace mxp {

__host__ __device__ static inline int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// ================================================================ preconditioner
__global__ __launch_bounds__(256) void k_scale_rows(int64_t n, const double* __restrict__ S, const double* __restrict__ V,
                                                    int64_t ldv, double* __restrict__ W, int nr) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int r = 0; r < nr; ++r) W[i + r * n] = S[i] * V[i + r * ldv];
}

__global__ __launch_bounds__(256) void k_copy_cols(int64_t n, const double* __restrict__ W, double* __restrict__ Z,
                                                   int64_t ldz, int nr) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int r = 0; r < nr; ++r) Z[i + r * ldz] = W[i + r * n];
}

// Diagonal-block solve with the full FP32 inverse: Y[k:k+kb] = Inv_k R[k:k+kb]
// (FP64 arithmetic).  Work-group = 64 rows; its 4 waves split the columns and
// their partial sums are added in a fixed order.  blockIdx.y = right-hand side.
__global__ __launch_bounds__(256) void k_prec_diag(int64_t n, int64_t k, int kb, int nb, const float* __restrict__ inv,
                                                   const double* __restrict__ R, double* __restrict__ Y) {
    __shared__ double part[4][64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int row = blockIdx.x * 64 + lane;
    const double* rhs = R + (int64_t)blockIdx.y * n + k;
    const int q = (kb + 3) / 4;
    const int c0 = wv * q, c1 = (c0 + q < kb) ? c0 + q : kb;
    double acc = 0.0;
    if (row < kb) {
        const float* col = inv + row;
#pragma unroll 8
        for (int c = c0; c < c1; ++c) acc += (double)col[(int64_t)c * nb] * rhs[c];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && row < kb) Y[(int64_t)blockIdx.y * n + k + row] = (part[0][lane] + part[1][lane]) +
                                                                    (part[2][lane] + part[3][lane]);
}

// Panel update R[rows] -= P z with z = Y[k:k+kb]: lower, rows k+kb..n-1 of
// L21 (each stored 32-row strip divided by its scale); upper, rows 0..k-1 of
// the U12 blocks above the diagonal block.  Thread = 2 consecutive rows; the
// 4 waves split the kb columns; partials added in a fixed order.
template <int ST, bool LOWER>
__global__ __launch_bounds__(256) void k_prec_panel(int64_t n, int64_t k, int kb, const typename Store<ST>::T* A,
                                                    int64_t lda, const float* __restrict__ lsc_blk,
                                                    const double* __restrict__ Y, double* __restrict__ R) {
    __shared__ double z[1024];
    __shared__ double part[4][128];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double* y = Y + (int64_t)blockIdx.y * n + k;
    double* rhs = R + (int64_t)blockIdx.y * n;
    for (int i = tid; i < kb; i += 256) z[i] = y[i];
    __syncthreads();
    const int64_t rbeg = LOWER ? k + kb : 0, rend = LOWER ? n : k;
    const int64_t row = rbeg + (int64_t)blockIdx.x * 128 + 2 * lane;
    const int q = (kb + 3) / 4;
    const int c0 = wv * q, c1 = (c0 + q < kb) ? c0 + q : kb;
    double a0 = 0.0, a1 = 0.0;
    if (row + 1 < rend) {
        const typename Store<ST>::T* p = A + row + k * lda;
#pragma unroll 8
        for (int c = c0; c < c1; ++c) {
            const int64_t o = (int64_t)c * lda;
            a0 += (double)Store<ST>::load(p, o) * z[c];
            a1 += (double)Store<ST>::load(p, o + 1) * z[c];
        }
    } else if (row < rend) {
        const typename Store<ST>::T* p = A + row + k * lda;
        for (int c = c0; c < c1; ++c) a0 += (double)Store<ST>::load(p, (int64_t)c * lda) * z[c];
    }
    part[wv][2 * lane] = a0;
    part[wv][2 * lane + 1] = a1;
    __syncthreads();
    if (tid < 128) {
        const int64_t r = rbeg + (int64_t)blockIdx.x * 128 + tid;
        if (r < rend) {
            double t = (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
            if (LOWER) t /= (double)lsc_blk[r / 32];
            rhs[r] -= t;
        }
    }
}

template <int ST>
static hipError_t prec_typed(const PrecPlan& p, const double* V, int64_t ldv, double* Z, int64_t ldz, int nr,
                             double* W, hipStream_t s) {
    typedef typename Store<ST>::T T;
    const int64_t n = p.n, nb = p.nb;
    const int64_t nblk = (n + nb - 1) / nb;
    const int64_t nstrips_total = (n + 31) / 32;
    double* R = W;                 // right-hand side, updated by the panels
    double* Y = W + n * nr;        // forward result, then the backward right-hand side
    unsigned rows_g = (unsigned)((n + 255) / 256);
    hipEvent_t pt = prof::begin(s);
    k_scale_rows<<<rows_g, 256, 0, s>>>(n, p.rowscale, V, ldv, R, nr);
    for (int64_t b = 0; b < nblk; ++b) {         // L y = S v
        int64_t k = b * nb;
        int kb = (int)(n - k < nb ? n - k : nb);
        k_prec_diag<<<dim3((unsigned)((kb + 63) / 64), nr), 256, 0, s>>>(n, k, kb, (int)nb, p.linv_full + b * nb * nb,
                                                                        R, Y);
        int64_t m = n - k - kb;
        if (m > 0)
            k_prec_panel<ST, true><<<dim3((unsigned)((m + 127) / 128), nr), 256, 0, s>>>(
                n, k, kb, (const T*)p.A, p.lda, p.lsc + b * nstrips_total, Y, R);
    }
    for (int64_t b = nblk - 1; b >= 0; --b) {    // U z = y
        int64_t k = b * nb;
        int kb = (int)(n - k < nb ? n - k : nb);
        k_prec_diag<<<dim3((unsigned)((kb + 63) / 64), nr), 256, 0, s>>>(n, k, kb, (int)nb, p.uinv_full + b * nb * nb,
                                                                        Y, R);
        if (k > 0)
            k_prec_panel<ST, false><<<dim3((unsigned)((k + 127) / 128), nr), 256, 0, s>>>(n, k, kb, (const T*)p.A,
                                                                                        p.lda, nullptr, R, Y);
    }
    k_copy_cols<<<rows_g, 256, 0, s>>>(n, R, Z, ldz, nr);
    prof::end(pt, prof::PREC, s, 2.0 * n * (double)n * nr, (double)n * n * sizeof(T) + 8.0 * n * nb);
    return hipGetLastError();
}

hipError_t prec_apply(const PrecPlan& p, const double* V, int64_t ldv, double* Z, int64_t ldz, int nr, double* W,
                      hipStream_t s) {
    switch (p.store) {
    case F32: return prec_typed<F32>(p, V, ldv, Z, ldz, nr, W, s);
    case F16: return prec_typed<F16>(p, V, ldv, Z, ldz, nr, W, s);
    case BF16: return prec_typed<BF16>(p, V, ldv, Z, ldz, nr, W, s);
    default: return hipErrorInvalidValue;
    }
}

// ================================================================ reductions
// Every reduction kernel gives block b the fixed index range
// [b*chunk, (b+1)*chunk) and sums it in a fixed order, so results are
// identical from run to run.
int red_blocks(int64_t n) {
    int64_t b = (n + 4095) / 4096;
    if (b > 256) b = 256;
    if (b < 1) b = 1;
    return (int)b;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
    v = warp_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

__device__ __forceinline__ double sum_parts(const double* part, int nparts, double* red) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) v += part[i];
    return block_sum(v, red);
}

// partial dot of x and y over the block's range
__global__ __launch_bounds__(256) void k_dot_part(int64_t n, int64_t chunk, const double* __restrict__ x,
                                                  const double* __restrict__ y, double* __restrict__ part) {
    __shared__ double red[4];
    int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    double v = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) v += x[i] * y[i];
    v = block_sum(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// MGS step j: h_j = sum(part_in); w -= h_j v_j over the block's range; then the
// partial dot for the next vector (v_{j+1} . w, or w . w after the last one).
__global__ __launch_bounds__(256) void k_mgs(int64_t n, int64_t chunk, const double* __restrict__ vj,
                                             const double* __restrict__ vnext, double* __restrict__ w,
                                             const double* __restrict__ part_in, double* __restrict__ part_out,
                                             double* __restrict__ hj) {
    __shared__ double red[4];
    double h = sum_parts(part_in, gridDim.x, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) *hj = h;
    int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    double v = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        double wi = w[i] - h * vj[i];
        w[i] = wi;
        v += (vnext ? vnext[i] : wi) * wi;
    }
    v = block_sum(v, red);
    if (threadIdx.x == 0) part_out[blockIdx.x] = v;
}

hipError_t mgs_step(int64_t n, const double* V, int k, double* w, double* hcol, double* part, hipStream_t s) {
    // V: n x (k+1) basis vectors v_0..v_k (column stride n); part: 2 x 256 scratch
    int nbk = red_blocks(n);
    int64_t chunk = (n + nbk - 1) / nbk;
    k_dot_part<<<nbk, 256, 0, s>>>(n, chunk, V, w, part);
    for (int j = 0; j <= k; ++j) {
        const double* vnext = (j < k) ? V + (int64_t)(j + 1) * n : nullptr;
        double* pin = part + (j & 1) * 256;
        double* pout = part + ((j + 1) & 1) * 256;
        k_mgs<<<nbk, 256, 0, s>>>(n, chunk, V + (int64_t)j * n, vnext, w, pin, pout, hcol + j);
    }
    return hipGetLastError();
}

// h = sqrt(sum(part)) ; v = w / h (v = 0 on exact breakdown)
__global__ __launch_bounds__(256) void k_normalize(int64_t n, int64_t chunk, const double* __restrict__ part,
                                                   const double* __restrict__ w, double* __restrict__ v,
                                                   double* __restrict__ hsub) {
    __shared__ double red[4];
    double h = sqrt(sum_parts(part, gridDim.x, red));
    if (blockIdx.x == 0 && threadIdx.x == 0) *hsub = h;
    int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) v[i] = (h > 0.0) ? w[i] / h : 0.0;
}

hipError_t norm_normalize(int64_t n, double* w, double* vout, double* hsub, double* part, hipStream_t s) {
    int nbk = red_blocks(n);
    int64_t chunk = (n + nbk - 1) / nbk;
    k_normalize<<<nbk, 256, 0, s>>>(n, chunk, part, w, vout, hsub);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ part, int nparts, double* out) {
    __shared__ double red[4];
    double v = sum_parts(part, nparts, red);
    if (threadIdx.x == 0) *out = sqrt(v);
}

hipError_t vec_norm2(int64_t n, const double* x, double* out, double* part, hipStream_t s) {
    int nbk = red_blocks(n);
    int64_t chunk = (n + nbk - 1) / nbk;
    k_dot_part<<<nbk, 256, 0, s>>>(n, chunk, x, x, part);
    k_norm_final<<<1, 256, 0, s>>>(part, nbk, out);
    return hipGetLastError();
}

// v = z / beta ; g[0] = beta
__global__ __launch_bounds__(256) void k_scale_copy(int64_t n, const double* __restrict__ z,
                                                    const double* __restrict__ beta, double* __restrict__ v,
                                                    double* __restrict__ g0) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double b = beta[0];
    if (i == 0) g0[0] = b;
    if (i < n) v[i] = (b > 0.0) ? z[i] / b : 0.0;
}

hipError_t vec_scale_copy(int64_t n, const double* x, const double* beta, double* v, double* g0, hipStream_t s) {
    k_scale_copy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, x, beta, v, g0);
    return hipGetLastError();
}

// ================================================================ Givens / least squares
// Column k of H (column-major, ldh): apply rotations 0..k-1, form rotation k
// that zeroes H[k+1,k], rotate g.  flag[0] = |g[k+1]|, flag[1] = 1 when
// |g[k+1]| <= tau * xnorm or H[k+1,k] was 0 (exact breakdown).
__global__ void k_givens(int k, double* H, int ldh, double* cs, double* sn, double* g, const double* xnorm,
                         double tau, double* flag) {
    if (threadIdx.x != 0) return;
    double* h = H + (int64_t)k * ldh;
    double hsub = h[k + 1];
    for (int i = 0; i < k; ++i) {
        double a = h[i], b = h[i + 1];
        h[i] = cs[i] * a + sn[i] * b;
        h[i + 1] = -sn[i] * a + cs[i] * b;
    }
    double a = h[k], b = h[k + 1];
    double rho = hypot(a, b);
    double c = (rho > 0.0) ? a / rho : 1.0, s = (rho > 0.0) ? b / rho : 0.0;
    cs[k] = c;
    sn[k] = s;
    h[k] = rho;
    h[k + 1] = 0.0;
    double gk = g[k];
    g[k + 1] = -s * gk;
    g[k] = c * gk;
    flag[0] = fabs(g[k + 1]);
    flag[1] = (fabs(g[k + 1]) <= tau * xnorm[0] || hsub == 0.0) ? 1.0 : 0.0;
}

hipError_t givens_step(int k, double* H, int ldh, double* cs, double* sn, double* g, const double* xnorm, double tau,
                       double* flag, hipStream_t s) {
    k_givens<<<1, 64, 0, s>>>(k, H, ldh, cs, sn, g, xnorm, tau, flag);
    return hipGetLastError();
}

// y = R^-1 g (R = rotated H[0:k, 0:k], upper triangular)
__global__ void k_backsub(int k, const double* H, int ldh, const double* g, double* y) {
    if (threadIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int l = i + 1; l < k; ++l) t -= H[i + (int64_t)l * ldh] * y[l];
        y[i] = t / H[i + (int64_t)i * ldh];
    }
}

// x += V[:, 0:k] y
__global__ __launch_bounds__(256) void k_axpy_basis(int64_t n, int k, const double* __restrict__ V,
                                                    const double* __restrict__ y, double* __restrict__ x) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += y[j] * V[i + (int64_t)j * n];
    x[i] += acc;
}

hipError_t lsq_update(int64_t n, int k, const double* H, int ldh, const double* g, double* y, const double* V,
                      double* x, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    k_backsub<<<1, 64, 0, s>>>(k, H, ldh, g, y);
    k_axpy_basis<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, k, V, y, x);
    return hipGetLastError();
}

}  // namespace mxp
