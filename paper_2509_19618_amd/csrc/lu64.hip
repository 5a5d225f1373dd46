// lu64.hip -- blocked LU in FP64 on the FP64 matrix cores, with or without
// partial pivoting, and the matching triangular solves.
//
// Two uses (paper: "Background" -- the figure of merit is measured against
// the FP64 solve of HPL; "Experimental Results" -- the pivoting study of
// Figures 2-4, LU in 64-bit arithmetic with and without partial pivoting):
//   * the FP64 baseline of the mixed-precision solve (same GPU, same timer);
//   * the largest pivot and the residual norms of FP64 LU with and without
//     partial pivoting on matrices with entries uniform in [-1, 1).
//
// Right-looking, block size nb (64 or 128).  Per block step k, m = n - k:
//   without pivoting: the nb x nb diagonal block is factored by one
//     work-group in LDS (k_diag64); L21 = A21 U11^-1 (k_trsm64_right) and
//     U12 = L11^-1 A12 (k_trsm64_left) by substitution, one column / row
//     per thread;
//   with pivoting: the m x nb panel is factored by one cooperative launch
//     (k_panel64_pp): every work-group holds a slice of the panel's rows in
//     LDS; per column each proposes its largest-magnitude candidate, a grid
//     barrier, every work-group picks the same winner (largest magnitude,
//     smallest row among equals -- the rule of LAPACK's getrf), the two rows
//     trade places and every work-group eliminates its rows.  The swaps are
//     then applied to the columns left and right of the panel (k_laswp64)
//     and U12 formed as above;
//   both: A22 <- A22 - L21 U12 with v_mfma_f64_16x16x4f64 (k_gemm64).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <mutex>

#include "../../include/mxp.h"
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace mxp {

typedef double d4v __attribute__((ext_vector_type(4)));

// ============================================================== trailing update
// C (M x N, ldc) -= A (M x K, lda) B (K x N, ldb), all column-major FP64.
// Work-group tile 128 x 128, four waves of 64 x 64 (4 x 4 blocks of the
// 16 x 16 MFMA).  Lane l of an MFMA supplies A[l%16][l/16] and B[l/16][l%16]
// of a 16 x 4 by 4 x 16 step and holds D[l/16 + 4q][l%16], q < 4.  The
// operands are read straight from memory (the FP64 matrix cores consume
// 16 bytes per lane per 64 cycles, which the L2 keeps up with); the next
// step's operands are loaded while the current one is multiplied.
constexpr int G64_T = 128;

__global__ __launch_bounds__(256) void k_gemm64(double* __restrict__ C, int64_t ldc, const double* __restrict__ A,
                                                int64_t lda, const double* __restrict__ B, int64_t ldb, int64_t M,
                                                int64_t N, int K) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * G64_T + wm * 64;
    const int64_t col0 = (int64_t)blockIdx.y * G64_T + wn * 64;
    // clamped operand addresses (rows / columns past the edge read a valid
    // element; their products land in results that are not stored)
    const double* ap[4];
    const double* bp[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int64_t r = row0 + a * 16 + li;
        r = r < M ? r : M - 1;
        ap[a] = A + r + (int64_t)lk * lda;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        int64_t c = col0 + b * 16 + li;
        c = c < N ? c : N - 1;
        bp[b] = B + lk + c * ldb;
    }
    d4v acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
    double fa[4], fb[4], na[4], nb_[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) fa[a] = ap[a][0];
#pragma unroll
    for (int b = 0; b < 4; ++b) fb[b] = bp[b][0];
    for (int k = 0; k < K; k += 4) {
        const int kn = k + 4 < K ? k + 4 : k;
#pragma unroll
        for (int a = 0; a < 4; ++a) na[a] = ap[a][(int64_t)kn * lda];
#pragma unroll
        for (int b = 0; b < 4; ++b) nb_[b] = bp[b][kn];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 4; ++a) fa[a] = na[a];
#pragma unroll
        for (int b = 0; b < 4; ++b) fb[b] = nb_[b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t c = col0 + b * 16 + li;
            if (c >= N) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = row0 + a * 16 + lk + 4 * q;
                if (r < M) C[r + c * ldc] -= acc[a][b][q];
            }
        }
}

hipError_t gemm64(double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                  int64_t N, int K, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (K % 4) return hipErrorInvalidValue;
    dim3 g((unsigned)((M + G64_T - 1) / G64_T), (unsigned)((N + G64_T - 1) / G64_T));
    hipEvent_t pt = prof::begin(prof::GEMM64, s);
    k_gemm64<<<g, 256, 0, s>>>(C, ldc, A, lda, B, ldb, M, N, K);
    prof::end(pt, prof::GEMM64, s, 2.0 * M * (double)N * K, 16.0 * M * (double)N + 8.0 * (M + N) * K);
    return hipGetLastError();
}

// The same update by rocBLAS's dgemm (a plain library GEMM), for the FP64
// baseline at the speed of the vendor library.  One handle per device; the
// stream is set and the call enqueued under a lock (a handle holds one
// stream at a time).
static std::mutex g_blas_mutex;
static rocblas_handle g_blas[64];

hipError_t gemm64_rocblas(double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb,
                          int64_t M, int64_t N, int K, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_blas_mutex);
    if (!g_blas[dev] && rocblas_create_handle(&g_blas[dev]) != rocblas_status_success) return hipErrorUnknown;
    if (rocblas_set_stream(g_blas[dev], s) != rocblas_status_success) return hipErrorUnknown;
    const double alpha = -1.0, beta = 1.0;
    hipEvent_t pt = prof::begin(prof::GEMM64, s);
    const rocblas_status st = rocblas_dgemm(g_blas[dev], rocblas_operation_none, rocblas_operation_none,
                                            (rocblas_int)M, (rocblas_int)N, (rocblas_int)K, &alpha, A,
                                            (rocblas_int)lda, B, (rocblas_int)ldb, &beta, C, (rocblas_int)ldc);
    prof::end(pt, prof::GEMM64, s, 2.0 * M * (double)N * K, 16.0 * M * (double)N + 8.0 * (M + N) * K);
    return st == rocblas_status_success ? hipSuccess : hipErrorUnknown;
}

// ============================================================== diagonal block (no pivoting)
// Unblocked right-looking LU of the kb x kb block at A[k, k] in LDS (kb <=
// 128: 128 KB), one work-group; a zero or non-finite pivot sets *info.
__global__ __launch_bounds__(256) void k_diag64(double* A, int64_t lda, int64_t k, int kb,
                                                unsigned long long* info) {
    extern __shared__ double D[];   // column-major, ld kb
    const int t = threadIdx.x;
    for (int e = t; e < kb * kb; e += 256) D[e] = A[(k + e % kb) + (k + e / kb) * lda];
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        const double piv = D[j + j * kb];
        const bool ok = piv != 0.0 && isfinite(piv);
        if (!ok && t == 0) atomicMin(info, (unsigned long long)(k + j + 1));
        if (ok) {
            const double rp = 1.0 / piv;
            for (int i = j + 1 + t; i < kb; i += 256) D[i + j * kb] *= rp;
        }
        __syncthreads();
        if (ok) {
            const int w = kb - j - 1;
            for (int e = t; e < w * w; e += 256) {
                const int i = j + 1 + e % w, c = j + 1 + e / w;
                D[i + c * kb] -= D[i + j * kb] * D[j + c * kb];
            }
        }
        __syncthreads();
    }
    for (int e = t; e < kb * kb; e += 256) A[(k + e % kb) + (k + e / kb) * lda] = D[e];
}

// ============================================================== triangular solves of a block step
// U12 = L11^-1 A12: one thread per column of A12 (nb values in LDS), forward
// substitution with the unit-lower L11 read as wave-uniform values.
constexpr int TW = 64;   // columns (rows) per work-group of the substitution kernels

__global__ __launch_bounds__(TW) void k_trsm64_left(double* A, int64_t lda, int64_t k, int nb, int64_t c_begin,
                                                    int64_t c_end) {
    extern __shared__ double X[];   // X[i * TW + t]
    const int t = threadIdx.x;
    const int64_t c0 = c_begin + (int64_t)blockIdx.x * TW;
    const int cols = (int)(c_end - c0 < TW ? c_end - c0 : TW);
    // coalesced load: the wave reads one column at a time
    for (int cc = 0; cc < cols; ++cc)
        for (int i = t; i < nb; i += TW) X[i * TW + cc] = A[(k + i) + (c0 + cc) * lda];
    __syncthreads();
    if (t < cols) {
        for (int i = 1; i < nb; ++i) {
            const double* Lrow = A + (k + i) + k * lda;   // L[i][p] = Lrow[p * lda]
            double s = X[i * TW + t];
            for (int p = 0; p < i; ++p) s -= Lrow[(int64_t)p * lda] * X[p * TW + t];
            X[i * TW + t] = s;
        }
    }
    __syncthreads();
    for (int cc = 0; cc < cols; ++cc)
        for (int i = t; i < nb; i += TW) A[(k + i) + (c0 + cc) * lda] = X[i * TW + cc];
}

// L21 = A21 U11^-1: one thread per row of A21, substitution against U11 by
// columns: x[j] = (a[j] - sum_{p<j} x[p] U[p][j]) / U[j][j].
__global__ __launch_bounds__(TW) void k_trsm64_right(double* A, int64_t lda, int64_t k, int nb, int64_t r_begin,
                                                     int64_t r_end) {
    extern __shared__ double X[];   // X[j * TW + t]
    const int t = threadIdx.x;
    const int64_t r0 = r_begin + (int64_t)blockIdx.x * TW;
    const int rows = (int)(r_end - r0 < TW ? r_end - r0 : TW);
    for (int j = 0; j < nb; ++j) X[j * TW + t] = (t < rows) ? A[(r0 + t) + (k + j) * lda] : 0.0;
    if (t < rows) {
        for (int j = 0; j < nb; ++j) {
            const double* Ucol = A + k + (k + j) * lda;   // U[p][j] = Ucol[p]
            double s = X[j * TW + t];
            for (int p = 0; p < j; ++p) s -= X[p * TW + t] * Ucol[p];
            X[j * TW + t] = s / Ucol[j];
        }
        for (int j = 0; j < nb; ++j) A[(r0 + t) + (k + j) * lda] = X[j * TW + t];
    }
}

// ============================================================== pivoted panel
// Grid barrier of a cooperative launch: bar[0] counts arrivals, bar[1] is
// the generation.  Release before the arrival, acquire after the wait; a
// bounded wait that expires sets *err and every work-group then stops.
__device__ bool grid_sync(unsigned* bar, unsigned nwg, int* err) {
    __shared__ int s_ok;
    // every wave's stores are released before the barrier (the work-group
    // barrier alone does not wait for them)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned old = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        if (old == nwg - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned it = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (++it > (1u << 24) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    atomicOr(err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

MXP_DEV void put64(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MXP_DEV double get64(const double* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// the better of two pivot candidates: larger magnitude, smaller row among equals
MXP_DEV void better(double& v, int64_t& r, double ov, int64_t orr) {
    if (ov > v || (ov == v && orr < r)) { v = ov; r = orr; }
}

// (value, row) maximum over the work-group (every thread gets the result)
MXP_DEV void wg_argmax(double& v, int64_t& r, double* redv, int64_t* redr) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) better(v, r, __shfl_xor(v, o, 64), __shfl_xor(r, o, 64));
    if (lane == 0) { redv[wv] = v; redr[wv] = r; }
    __syncthreads();
    v = redv[0];
    r = redr[0];
    for (int q = 1; q < 4; ++q) better(v, r, redv[q], redr[q]);
    __syncthreads();
}

// Panel columns [k, k+nb), rows [k, n): work-group w holds rows
// [k + w rpw, k + (w+1) rpw) in LDS (P[c * rpw + rr]), one row per thread.
// cand: 2 x nwg slots of (|value|, row, nb row values); top: 2 x nb (the
// current pivot position's row); both double-buffered by column parity.
__global__ __launch_bounds__(256) void k_panel64_pp(double* A, int64_t lda, int64_t n, int64_t k, int nb, int rpw,
                                                    int64_t* ipiv, double* cand, double* top, unsigned* bar,
                                                    unsigned long long* info, int* err) {
    extern __shared__ double P[];
    __shared__ double prow[128];
    __shared__ double redv[4];
    __shared__ int64_t redr[4];
    const int t = threadIdx.x;
    const unsigned nwg = gridDim.x;
    const int w = (int)blockIdx.x;
    const int64_t rbase = k + (int64_t)w * rpw;                 // global row of local row 0
    const int nrows = (int)(n - rbase < rpw ? n - rbase : rpw);
    const int slot = nb + 2;
    for (int c = 0; c < nb; ++c)
        if (t < nrows) P[c * rpw + t] = A[(rbase + t) + (k + c) * lda];
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        const int par = j & 1;
        const int64_t gtop = k + j;                            // pivot position
        // (a) this work-group's candidate: the largest |P[j][r]| on or below the pivot position
        double bv = -1.0;
        int64_t br = INT64_MAX;
        if (t < nrows && rbase + t >= gtop) {
            bv = fabs(P[j * rpw + t]);
            br = rbase + t;
        }
        wg_argmax(bv, br, redv, redr);
        double* my = cand + (int64_t)(par * nwg + w) * slot;
        if (t == 0) {
            put64(&my[0], bv);
            put64(&my[1], bv >= 0.0 ? (double)br : -1.0);
        }
        if (bv >= 0.0 && t < nb) put64(&my[2 + t], P[t * rpw + (int)(br - rbase)]);
        if (gtop >= rbase && gtop < rbase + nrows && t < nb) put64(&top[par * nb + t], P[t * rpw + (int)(gtop - rbase)]);
        // (b) every candidate and the top row are published
        if (!grid_sync(bar, nwg, err)) return;
        // (c) the winner, the same in every work-group: one candidate per thread
        double cv = -1.0;
        int64_t cr = INT64_MAX;
        if (t < (int)nwg) {
            const double* cq = cand + (int64_t)(par * nwg + t) * slot;
            const double v = get64(&cq[0]);
            const double r = get64(&cq[1]);
            if (r >= 0.0) { cv = v; cr = (int64_t)r; }
        }
        wg_argmax(cv, cr, redv, redr);
        const int64_t p = cr;
        if (w == 0 && t == 0) ipiv[gtop] = p;
        const int wp = (int)((p - k) / rpw);
        if (t < nb) prow[t] = get64(&cand[(int64_t)(par * nwg + wp) * slot + 2 + t]);
        __syncthreads();
        // (d) rows gtop and p trade places
        if (p != gtop) {
            if (p >= rbase && p < rbase + nrows && t < nb) P[t * rpw + (int)(p - rbase)] = get64(&top[par * nb + t]);
            if (gtop >= rbase && gtop < rbase + nrows && t < nb) P[t * rpw + (int)(gtop - rbase)] = prow[t];
        }
        __syncthreads();
        // (e) eliminate below the pivot
        const double piv = prow[j];
        const bool ok = piv != 0.0 && isfinite(piv);
        if (!ok && w == 0 && t == 0) atomicMin(info, (unsigned long long)(gtop + 1));
        if (ok && t < nrows && rbase + t > gtop) {
            const double l = P[j * rpw + t] / piv;
            P[j * rpw + t] = l;
            for (int c = j + 1; c < nb; ++c) P[c * rpw + t] -= l * prow[c];
        }
        __syncthreads();
    }
    for (int c = 0; c < nb; ++c)
        if (t < nrows) A[(rbase + t) + (k + c) * lda] = P[c * rpw + t];
}

// Row swaps ipiv[k .. k+nb) applied in order to the columns [c_begin, c_end)
// that are outside the panel: one thread per column.
__global__ __launch_bounds__(256) void k_laswp64(double* A, int64_t lda, const int64_t* __restrict__ ipiv, int64_t k,
                                                 int nb, int64_t c_begin, int64_t c_end) {
    const int64_t c = c_begin + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= c_end) return;
    double* col = A + c * lda;
    for (int j = 0; j < nb; ++j) {
        const int64_t p = ipiv[k + j];
        if (p != k + j) {
            const double x = col[k + j];
            col[k + j] = col[p];
            col[p] = x;
        }
    }
}

// ============================================================== solve
// x <- P x (the swaps in order), then unit-lower forward and upper backward
// substitution, blocked by 64 rows: per block one work-group solves the
// triangle (the block's 64 x 64 diagonal block in LDS), then every row
// below (above) subtracts the block's contribution (one thread per row).
__global__ void k_apply_pivots(double* x, int64_t ldx, int nr, const int64_t* __restrict__ ipiv, int64_t n) {
    const int r = threadIdx.x;
    if (r >= nr) return;
    double* v = x + r * ldx;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t p = ipiv[k];
        if (p != k) {
            const double a = v[k];
            v[k] = v[p];
            v[p] = a;
        }
    }
}

constexpr int SB = 64;

template <bool LOWER>
__global__ __launch_bounds__(64) void k_trsv64_block(const double* __restrict__ A, int64_t lda, int64_t n,
                                                     int64_t b0, double* x, int64_t ldx, int nr) {
    __shared__ double D[SB * SB];
    const int t = threadIdx.x;
    const int kb = (int)(n - b0 < SB ? n - b0 : SB);
    for (int c = 0; c < kb; ++c)
        if (t < kb) D[t + c * SB] = A[(b0 + t) + (b0 + c) * lda];
    __syncthreads();
    if (t < nr) {
        double* v = x + t * ldx + b0;
        if (LOWER) {
            for (int i = 1; i < kb; ++i) {
                double s = v[i];
                for (int p = 0; p < i; ++p) s -= D[i + p * SB] * v[p];
                v[i] = s;
            }
        } else {
            for (int i = kb - 1; i >= 0; --i) {
                double s = v[i];
                for (int p = i + 1; p < kb; ++p) s -= D[i + p * SB] * v[p];
                v[i] = s / D[i + i * SB];
            }
        }
    }
}

// rows [r_begin, r_end) -= A[rows, b0 : b0+kb] x[b0 : b0+kb]
__global__ __launch_bounds__(256) void k_gemv64_update(const double* __restrict__ A, int64_t lda, int64_t b0, int kb,
                                                       int64_t r_begin, int64_t r_end, double* x, int64_t ldx,
                                                       int nr) {
    const int64_t r = r_begin + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= r_end) return;
    for (int q = 0; q < nr; ++q) {
        const double* v = x + q * ldx + b0;
        double s = 0.0;
        for (int c = 0; c < kb; ++c) s += A[r + (b0 + c) * lda] * v[c];
        x[q * ldx + r] -= s;
    }
}

// ============================================================== drivers
int lu64_block(int64_t n) {
    // the pivoted panel holds ceil(m / 256) rows x nb per work-group in at most 128 KB of LDS
    const int64_t rpw = (n + 255) / 256;
    return rpw <= 128 ? 128 : 64;
}

size_t lu64_work_bytes(int64_t n) {
    const int nb = lu64_block(n);
    return (size_t)2 * 256 * (nb + 2) * 8 + (size_t)2 * nb * 8 + 256 + 64;
}

hipError_t lu64_factor(int64_t n, double* A, int64_t lda, int64_t* ipiv, void* work, unsigned long long* info_dev,
                       int use_rocblas, hipStream_t s) {
    const int nb = lu64_block(n);
    static const hipError_t attr = []() {
        hipError_t e;
        if ((e = hipFuncSetAttribute((const void*)k_diag64, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 128 * 8)))
            return e;
        if ((e = hipFuncSetAttribute((const void*)k_panel64_pp, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     128 * 1024)))
            return e;
        if ((e = hipFuncSetAttribute((const void*)k_trsm64_left, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     128 * TW * 8)))
            return e;
        return hipFuncSetAttribute((const void*)k_trsm64_right, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   128 * TW * 8);
    }();
    if (attr) return attr;
    char* wb = (char*)work;
    double* cand = (double*)wb;
    double* top = cand + 2 * 256 * (nb + 2);
    unsigned* bar = (unsigned*)(top + 2 * nb);
    int* err = (int*)(bar + 2);
    hipError_t e;
    if ((e = fill_u64(info_dev, 1, ~0ull, s))) return e;
    if ((e = fill_u64(bar, 2, 0ull, s))) return e;   // bar[0..1] and err
    for (int64_t k = 0; k < n; k += nb) {
        const int kb = (int)(n - k < nb ? n - k : nb);
        const int64_t m = n - k;
        if (ipiv) {
            int rpw = (int)((m + 255) / 256);
            if (rpw < 64) rpw = (int)(m < 64 ? m : 64);
            const unsigned nwg = (unsigned)((m + rpw - 1) / rpw);
            const size_t lds = (size_t)rpw * kb * 8;
            double* Ap = A;
            int64_t nn = n, kk = k;
            int kbv = kb, rpwv = rpw;
            void* args[] = {&Ap, (void*)&lda, &nn, &kk, &kbv, &rpwv, &ipiv, &cand, &top, &bar, &info_dev, &err};
            if ((e = hipLaunchCooperativeKernel((const void*)k_panel64_pp, dim3(nwg), dim3(256), args, (unsigned)lds,
                                                s)))
                return e;
            // the swaps, left and right of the panel
            if (k > 0) k_laswp64<<<(unsigned)((k + 255) / 256), 256, 0, s>>>(A, lda, ipiv, k, kb, 0, k);
            if (k + kb < n)
                k_laswp64<<<(unsigned)((n - k - kb + 255) / 256), 256, 0, s>>>(A, lda, ipiv, k, kb, k + kb, n);
        } else {
            k_diag64<<<1, 256, (size_t)kb * kb * 8, s>>>(A, lda, k, kb, info_dev);
            if (k + kb < n)
                k_trsm64_right<<<(unsigned)((n - k - kb + TW - 1) / TW), TW, (size_t)kb * TW * 8, s>>>(
                    A, lda, k, kb, k + kb, n);
        }
        if ((e = hipGetLastError())) return e;
        if (k + kb < n) {
            k_trsm64_left<<<(unsigned)((n - k - kb + TW - 1) / TW), TW, (size_t)kb * TW * 8, s>>>(A, lda, k, kb,
                                                                                              k + kb, n);
            if ((e = hipGetLastError())) return e;
            auto g64 = use_rocblas ? gemm64_rocblas : gemm64;
            if ((e = g64(A + (k + kb) + (k + kb) * lda, lda, A + (k + kb) + k * lda, lda, A + k + (k + kb) * lda, lda,
                         m - kb, m - kb, kb, s)))
                return e;
        }
    }
    return hipSuccess;
}

int* lu64_err_word(void* work, int64_t n) {
    const int nb = lu64_block(n);
    double* cand = (double*)work;
    double* top = cand + 2 * 256 * (nb + 2);
    return (int*)((unsigned*)(top + 2 * nb) + 2);
}

hipError_t lu64_solve(int64_t n, const double* A, int64_t lda, const int64_t* ipiv, double* X, int64_t ldx, int nr,
                      hipStream_t s) {
    hipError_t e;
    if (ipiv) {
        k_apply_pivots<<<1, 64, 0, s>>>(X, ldx, nr, ipiv, n);
        if ((e = hipGetLastError())) return e;
    }
    for (int64_t b0 = 0; b0 < n; b0 += SB) {
        const int kb = (int)(n - b0 < SB ? n - b0 : SB);
        k_trsv64_block<true><<<1, 64, 0, s>>>(A, lda, n, b0, X, ldx, nr);
        if (b0 + kb < n)
            k_gemv64_update<<<(unsigned)((n - b0 - kb + 255) / 256), 256, 0, s>>>(A, lda, b0, kb, b0 + kb, n, X, ldx,
                                                                                  nr);
    }
    for (int64_t b0 = (n - 1) / SB * SB; b0 >= 0; b0 -= SB) {
        const int kb = (int)(n - b0 < SB ? n - b0 : SB);
        k_trsv64_block<false><<<1, 64, 0, s>>>(A, lda, n, b0, X, ldx, nr);
        if (b0 > 0) k_gemv64_update<<<(unsigned)((b0 + 255) / 256), 256, 0, s>>>(A, lda, b0, kb, 0, b0, X, ldx, nr);
    }
    return hipGetLastError();
}

}  // namespace mxp
