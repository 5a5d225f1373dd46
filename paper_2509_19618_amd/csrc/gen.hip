// gen.hip -- counter-based matrix generation and the FP64 residual that
// regenerates the matrix instead of reading it (paper: "Matrix Generation",
// scalable generation with any entry computable on its own; "Algorithmic
// Framework", 64-bit residual of the refinement and the HPL scaled residual).
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace mxp {

// ---------------------------------------------------------------- fills
__global__ void k_fill_u64(uint64_t* p, int64_t count, uint64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

hipError_t fill_u64(void* p, int64_t count, uint64_t v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill_u64<<<dim3((unsigned)blocks), dim3(256), 0, s>>>((uint64_t*)p, count, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------- generation
// Thread (row i, column quad q): one Philox call gives A[i, 4q..4q+3].
// Each thread also accumulates sum_j |k(i,j) - 2^31| exactly in 64-bit
// integers; the per-row sums are combined with integer atomics, which are
// exact and order independent.  Entries are s 2^-32 (s = k - 2^31) for the
// matrices with entries in [-1/2, 1/2), s 2^-31 for those in [-1, 1).
constexpr int GEN_QUADS = 64;  // column quads per thread

template <int ST>
__global__ __launch_bounds__(256) void k_gen_matrix(int64_t n, uint64_t seed, double scale,
                                                    typename Store<ST>::T* A, int64_t lda,
                                                    unsigned long long* rowsum) {
    uint32_t k0[10], k1[10];
    philox_keys(seed, k0, k1);
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int64_t q0 = (int64_t)blockIdx.y * GEN_QUADS;
    int64_t nq = (n + 3) / 4;
    int64_t q1 = q0 + GEN_QUADS < nq ? q0 + GEN_QUADS : nq;
    unsigned long long acc = 0;
    for (int64_t q = q0; q < q1; ++q) {
        uint32_t w[4];
        philox4((uint32_t)i, (uint32_t)q, 0u, k0, k1, w);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int64_t j = 4 * q + t;
            if (j < n) {
                int32_t s = draw_offset(w[t]);
                acc += (unsigned long long)(s < 0 ? -(int64_t)s : (int64_t)s);
                if (A) A[i + j * lda] = Store<ST>::from_f64((double)s * scale);
            }
        }
    }
    atomicAdd(&rowsum[i], acc);
}

// The diagonal and the row 1-norms from the integer row sums S (held in the
// diag array until here) and the row's own draw s_ii:
//   dominant: A_ii = S 2^-32 (the whole row's |draws|, own one included),
//             ||A_i||_1 = (2S - |s_ii|) 2^-32;
//   sqrt(n):  A_ii = s_ii 2^-32 + shift (shift = gamma sqrt(n), formed on the
//             host), ||A_i||_1 = (S - |s_ii|) 2^-32 + |A_ii|;
//   uniform:  A_ii = s_ii 2^-31, ||A_i||_1 = S 2^-31.
// ||A||_inf is the largest row norm: a maximum over the bit patterns of
// non-negative doubles, which order like the values.
template <int ST>
__global__ __launch_bounds__(256) void k_gen_finalize(int64_t n, uint64_t seed, int kind, double shift,
                                                      typename Store<ST>::T* A, int64_t lda, double* diag,
                                                      double* row_l1, unsigned long long* amax) {
    uint32_t k0[10], k1[10];
    philox_keys(seed, k0, k1);
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    unsigned long long S = ((const unsigned long long*)diag)[i];
    uint32_t w[4];
    philox4((uint32_t)i, (uint32_t)(i >> 2), 0u, k0, k1, w);
    int32_t s = draw_offset(w[i & 3]);
    unsigned long long own = (unsigned long long)(s < 0 ? -(int64_t)s : (int64_t)s);
    double d, l1;
    if (kind == 1) {
        d = (double)s * 0x1p-32 + shift;
        l1 = (double)(S - own) * 0x1p-32 + fabs(d);
    } else if (kind == 2) {
        d = (double)s * 0x1p-31;
        l1 = (double)S * 0x1p-31;
    } else {
        d = (double)S * 0x1p-32;
        l1 = (double)(2ull * S - own) * 0x1p-32;
    }
    diag[i] = d;
    if (row_l1) row_l1[i] = l1;
    if (A) A[i + i * lda] = Store<ST>::from_f64(d);
    atomicMax(amax, (unsigned long long)__double_as_longlong(l1));
}

__global__ void k_gen_anorm(double* a_inf) {
    unsigned long long m = *(unsigned long long*)a_inf;
    *a_inf = __longlong_as_double((long long)m);
}

__global__ __launch_bounds__(256) void k_gen_rhs(int64_t n, int64_t nrhs, uint64_t seed, double* B, int64_t ldb) {
    uint32_t k0[10], k1[10];
    philox_keys(seed, k0, k1);
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int64_t q = 0; q < (nrhs + 3) / 4; ++q) {
        uint32_t w[4];
        philox4((uint32_t)i, (uint32_t)q, 1u, k0, k1, w);
        for (int t = 0; t < 4; ++t) {
            int64_t r = 4 * q + t;
            if (r < nrhs) B[i + r * ldb] = draw_value(w[t]);
        }
    }
}

double gen_offscale(int kind) { return kind == 2 ? 0x1p-31 : 0x1p-32; }

template <int ST>
static hipError_t gen_launch(int64_t n, int64_t nrhs, uint64_t seed, int kind, double shift, void* A, int64_t lda,
                             double* B, int64_t ldb, double* diag, double* row_l1, double* a_inf, hipStream_t s) {
    typedef typename Store<ST>::T T;
    hipError_t e;
    if ((e = fill_u64(diag, n, 0, s))) return e;
    if ((e = fill_u64(a_inf, 1, 0, s))) return e;
    dim3 g((unsigned)((n + 255) / 256), (unsigned)(((n + 3) / 4 + GEN_QUADS - 1) / GEN_QUADS));
    k_gen_matrix<ST><<<g, dim3(256), 0, s>>>(n, seed, gen_offscale(kind), (T*)A, lda, (unsigned long long*)diag);
    if ((e = hipGetLastError())) return e;
    k_gen_finalize<ST><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, seed, kind, shift, (T*)A, lda,
                                                                               diag, row_l1,
                                                                               (unsigned long long*)a_inf);
    if ((e = hipGetLastError())) return e;
    k_gen_anorm<<<1, 1, 0, s>>>(a_inf);
    if ((e = hipGetLastError())) return e;
    if (nrhs > 0 && B) {
        k_gen_rhs<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, nrhs, seed, B, ldb);
        if ((e = hipGetLastError())) return e;
    }
    return hipSuccess;
}

hipError_t generate(int64_t n, int64_t nrhs, uint64_t seed, int kind, double shift, int store, void* A, int64_t lda,
                    double* B, int64_t ldb, double* diag, double* row_l1, double* a_inf, hipStream_t s) {
    switch (store) {
    case F64: return gen_launch<F64>(n, nrhs, seed, kind, shift, A, lda, B, ldb, diag, row_l1, a_inf, s);
    case F32: return gen_launch<F32>(n, nrhs, seed, kind, shift, A, lda, B, ldb, diag, row_l1, a_inf, s);
    case F16: return gen_launch<F16>(n, nrhs, seed, kind, shift, A, lda, B, ldb, diag, row_l1, a_inf, s);
    case BF16: return gen_launch<BF16>(n, nrhs, seed, kind, shift, A, lda, B, ldb, diag, row_l1, a_inf, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- regenerating GEMV
// Partial products P[c][r][i] = sum over the columns j of chunk c, j != i,
// of A[i,j] * X[j,r], with A[i,j] regenerated.  A thread owns one row; all
// threads of a wave walk the same columns, so X[j,r] is a wave-uniform load.
// The sums are taken over the integer draws s (A[i,j] = s 2^-32) and scaled
// by the power of two of the matrix kind (2^-32, or 2^-31 for entries in
// [-1, 1)) once at the end: scaling by a power of two commutes with every
// rounding, so the result is that of summing the draws' values.  The sign
// flip of the draws (s = word ^ 2^31) is folded into the last round keys for
// words 0 and 2, which leave the last round xor-ed with them (the caller
// passes those keys flipped); words 1 and 3 are flipped here.  Chunks start
// at multiples of four columns; full quads of columns run without bound
// checks, and the diagonal test is compiled in only for the work-groups
// whose rows meet the chunk's columns.
template <int NR, bool DIAG>
MXP_DEV void regen_cols(uint32_t row, int64_t i, int64_t j0, int64_t j1, const uint32_t k0[10],
                        const uint32_t k1[10], const double* __restrict__ X, int64_t ldx, double acc[NR]) {
    const int64_t jq = j0 + ((j1 - j0) & ~(int64_t)3);
    for (int64_t j = j0; j < jq; j += 4) {
        uint32_t w[4];
        philox4(row, (uint32_t)(j >> 2), 0u, k0, k1, w);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double a = (double)(int32_t)(w[t] ^ ((t & 1) ? 0x80000000u : 0u));
            if (DIAG) a = ((uint32_t)(j + t) == (uint32_t)i) ? 0.0 : a;
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r] = fma(a, X[j + t + r * ldx], acc[r]);
        }
    }
    if (jq < j1) {
        uint32_t w[4];
        philox4(row, (uint32_t)(jq >> 2), 0u, k0, k1, w);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int64_t jj = jq + t;
            if (jj < j1) {
                double a = (double)(int32_t)(w[t] ^ ((t & 1) ? 0x80000000u : 0u));
                a = (jj == i) ? 0.0 : a;
#pragma unroll
                for (int r = 0; r < NR; ++r) acc[r] = fma(a, X[jj + r * ldx], acc[r]);
            }
        }
    }
}

template <int NR>
__global__ __launch_bounds__(256) void k_regen_gemv(int64_t n, uint64_t seed, double offscale,
                                                    const double* __restrict__ X, int64_t ldx,
                                                    double* __restrict__ P, int64_t chunk_cols) {
    uint32_t k0[10], k1[10];
    philox_keys(seed, k0, k1);
    k0[9] ^= 0x80000000u;                     // sign flip of words 0 and 2
    k1[9] ^= 0x80000000u;
    const int64_t r_lo = (int64_t)blockIdx.x * 256;
    const int64_t i = r_lo + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * chunk_cols;
    const int64_t j1 = j0 + chunk_cols < n ? j0 + chunk_cols : n;
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    const uint32_t row = (uint32_t)(i < n ? i : 0);
    if (r_lo < j1 && j0 < r_lo + 256) regen_cols<NR, true>(row, i, j0, j1, k0, k1, X, ldx, acc);
    else regen_cols<NR, false>(row, i, j0, j1, k0, k1, X, ldx, acc);
    if (i < n) {
#pragma unroll
        for (int r = 0; r < NR; ++r) P[((int64_t)blockIdx.y * NR + r) * n + i] = acc[r] * offscale;
    }
}

// R[i,r] = B[i,r] - (diag[i] X[i,r] + sum_c P[c][r][i]) (or without B: R = A X),
// chunks summed in a fixed order so the result is run-to-run identical.
__global__ __launch_bounds__(256) void k_regen_reduce(int64_t n, int nr, int64_t nchunk, const double* __restrict__ P,
                                                      const double* __restrict__ diag, const double* __restrict__ X,
                                                      int64_t ldx, const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ R, int64_t ldr) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int r = 0; r < nr; ++r) {
        double s = diag[i] * X[i + r * ldx];
        for (int64_t c = 0; c < nchunk; ++c) s += P[(c * nr + r) * n + i];
        R[i + r * ldr] = B ? B[i + r * ldb] - s : s;
    }
}

int64_t regen_chunk_cols(int64_t n) {
    // enough column chunks to give the GPU >= ~2048 workgroups
    int64_t row_tiles = (n + 255) / 256;
    int64_t want = (2048 + row_tiles - 1) / row_tiles;
    int64_t cc = (n + want - 1) / want;
    cc = (cc + 63) / 64 * 64;
    if (cc < 256) cc = 256;
    return cc;
}

size_t regen_partial_bytes(int64_t n, int nr) {
    int64_t cc = regen_chunk_cols(n);
    int64_t nchunk = (n + cc - 1) / cc;
    return (size_t)nchunk * nr * n * sizeof(double);
}

hipError_t regen_matvec(int64_t n, uint64_t seed, int kind, const double* diag, const double* X, int64_t ldx, int nr,
                        const double* B, int64_t ldb, double* R, int64_t ldr, double* P, hipStream_t s) {
    const double osc = gen_offscale(kind);
    int64_t cc = regen_chunk_cols(n);
    int64_t nchunk = (n + cc - 1) / cc;
    dim3 g((unsigned)((n + 255) / 256), (unsigned)nchunk);
    // the column loop steps by 4 from a chunk start that is a multiple of 4
    hipEvent_t pt = prof::begin(prof::REGEN, s);
    for (int r0 = 0; r0 < nr;) {
        int left = nr - r0;
        int w = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
        switch (w) {
        case 8: k_regen_gemv<8><<<g, dim3(256), 0, s>>>(n, seed, osc, X + r0 * ldx, ldx, P, cc); break;
        case 4: k_regen_gemv<4><<<g, dim3(256), 0, s>>>(n, seed, osc, X + r0 * ldx, ldx, P, cc); break;
        case 2: k_regen_gemv<2><<<g, dim3(256), 0, s>>>(n, seed, osc, X + r0 * ldx, ldx, P, cc); break;
        default: k_regen_gemv<1><<<g, dim3(256), 0, s>>>(n, seed, osc, X + r0 * ldx, ldx, P, cc); break;
        }
        hipError_t e = hipGetLastError();
        if (e) return e;
        k_regen_reduce<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(
            n, w, nchunk, P, diag, X + r0 * ldx, ldx, B ? B + r0 * ldb : nullptr, ldb, R + r0 * ldr, ldr);
        if ((e = hipGetLastError())) return e;
        r0 += w;
    }
    prof::end(pt, prof::REGEN, s, 2.0 * n * (double)n * nr, 16.0 * n * nr + 8.0 * n * nchunk * nr);
    return hipSuccess;
}

// ---------------------------------------------------------------- norms
// Per-block maxima of |r|, |x|, |b| (three columns of partials) for each
// right-hand side q = blockIdx.y, then one block per right-hand side forms
// eta = ||r|| / ((||A|| ||x|| + ||b||) n 2^-53).
__global__ __launch_bounds__(256) void k_absmax3(int64_t n, const double* __restrict__ r, int64_t ldr,
                                                 const double* __restrict__ x, int64_t ldx,
                                                 const double* __restrict__ b, int64_t ldb,
                                                 double* __restrict__ part) {
    __shared__ double red[3][4];
    const int q = blockIdx.y;
    r += q * ldr;
    x += q * ldx;
    b += q * ldb;
    part += (int64_t)q * gridDim.x * 3;
    double mr = 0, mx = 0, mb = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        mr = fmax(mr, fabs(r[i]));
        mx = fmax(mx, fabs(x[i]));
        mb = fmax(mb, fabs(b[i]));
    }
    mr = warp_max(mr); mx = warp_max(mx); mb = warp_max(mb);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = mr; red[1][w] = mx; red[2][w] = mb; }
    __syncthreads();
    if (threadIdx.x < 3) {
        double m = fmax(fmax(red[threadIdx.x][0], red[threadIdx.x][1]), fmax(red[threadIdx.x][2], red[threadIdx.x][3]));
        part[blockIdx.x * 3 + threadIdx.x] = m;
    }
}

// eta_out[4 q .. 4 q + 2] = (eta, ||x||_inf, ||r||_inf) of right-hand side q
__global__ void k_eta_final(int64_t n, int nblk, const double* __restrict__ part, const double* __restrict__ a_inf,
                            double* __restrict__ eta_out) {
    __shared__ double red[3][4];
    const int q = blockIdx.x;
    part += (int64_t)q * nblk * 3;
    double mr = 0, mx = 0, mb = 0;
    for (int i = threadIdx.x; i < nblk; i += 256) {
        mr = fmax(mr, part[i * 3 + 0]);
        mx = fmax(mx, part[i * 3 + 1]);
        mb = fmax(mb, part[i * 3 + 2]);
    }
    mr = warp_max(mr); mx = warp_max(mx); mb = warp_max(mb);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = mr; red[1][w] = mx; red[2][w] = mb; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double R = 0, Xn = 0, Bn = 0;
        for (int k = 0; k < 4; ++k) { R = fmax(R, red[0][k]); Xn = fmax(Xn, red[1][k]); Bn = fmax(Bn, red[2][k]); }
        double den = (a_inf[0] * Xn + Bn) * (double)n * 0x1p-53;
        eta_out[4 * q] = R / den;
        eta_out[4 * q + 1] = Xn;
        eta_out[4 * q + 2] = R;
    }
}

int eta_blocks(int64_t n) {
    int64_t b = (n + 2047) / 2048;
    if (b > 512) b = 512;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t hpl_eta_dev(int64_t n, int nr, const double* r, int64_t ldr, const double* x, int64_t ldx,
                       const double* b, int64_t ldb, const double* a_inf, double* part, double* eta_out,
                       hipStream_t s) {
    int nb = eta_blocks(n);
    k_absmax3<<<dim3(nb, nr), dim3(256), 0, s>>>(n, r, ldr, x, ldx, b, ldb, part);
    hipError_t e = hipGetLastError();
    if (e) return e;
    k_eta_final<<<nr, 256, 0, s>>>(n, nb, part, a_inf, eta_out);
    return hipGetLastError();
}

}  // namespace mxp

namespace mxp {

// ---------------------------------------------------------------- residual without allocation
// For callers that cannot allocate (code under stream capture, tight serving
// loops): the partial products of the regenerating GEMV live in a file-scope
// device array instead of a work buffer.  Its host-side name is not a device
// address: the address is looked up once per device and kept.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(32) << 20;
static __device__ __align__(256) double scratch[STATIC_SCRATCH_BYTES / sizeof(double)];

static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[64];

hipError_t static_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)))) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t static_scratch_bytes() { return STATIC_SCRATCH_BYTES; }

}  // namespace mxp
