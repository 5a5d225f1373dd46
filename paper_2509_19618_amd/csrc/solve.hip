// solve.hip -- FP64 pieces of the GMRES-based refinement (paper:
// "Algorithmic Framework": the low-precision factors used as a left
// preconditioner, GMRES in 64-bit, at most 50 iterations).
//
// prec_apply: z = U^-1 L^-1 S v by block forward and backward substitution
// on the stored factor (FP64 arithmetic): the nb x nb diagonal blocks are
// applied through the full FP32 inverses kept by the factorisation, the
// off-diagonal panels are read in the storage format (L21 strips unscaled by
// their power-of-two factor); one dataflow kernel per triangular solve.
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

// ---------------------------------------------------------------- block substitution
// One kernel per triangular solve.  Work-group = one strip of TS rows; strips
// are processed as a dataflow: a strip of block j accumulates the products of
// its rows of the off-diagonal factor with every dependency block's solution
// as soon as that block is published (flag `ready`), then the strips of block
// j meet (flag `cnt`) and each applies its rows of the FP32 inverse of the
// diagonal block and publishes them.  Forward (L): dependencies are the blocks
// before j, strips run in increasing order; backward (U): the blocks after j,
// strips in decreasing order.  Work-groups are dispatched in index order and
// every wait is on a strip of smaller index (or of the same block), so the
// chain always progresses; each wait is still bounded and on expiry sets
// *err and lets the work-group exit.  All sums are taken in a fixed order
// (deterministic results).
constexpr int TS = 64;

// Values exchanged between work-groups (block solutions, block right-hand
// sides) are written and read with device-scope atomic accesses, which go to
// the device's coherence point instead of an XCD's L2; a flag is raised only
// after every wave has its stores acknowledged, so no cache write-back or
// invalidation is needed.
MXP_DEV void put_shared(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MXP_DEV double get_shared(const double* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// v, treated as written at this point: arithmetic on prefetched registers
// cannot move above it (the compiler would otherwise unpack a load's result
// right after issuing it, which waits for the load)
MXP_DEV void pin4(uint4& v) { asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w)); }
MXP_DEV void pin4f(float4& v) { asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w)); }

// element k of a 16-byte vector of storage values, taken from its 32-bit
// words (no access through a cast pointer, which would split the vector at
// its load)
template <int ST> MXP_DEV float u4_elem(const uint4& v, int k);
template <> MXP_DEV float u4_elem<F32>(const uint4& v, int k) {
    const unsigned w[4] = {v.x, v.y, v.z, v.w};
    return __uint_as_float(w[k]);
}
template <> MXP_DEV float u4_elem<F16>(const uint4& v, int k) {
    const unsigned w[4] = {v.x, v.y, v.z, v.w};
    const unsigned h = (k & 1) ? (w[k >> 1] >> 16) : (w[k >> 1] & 0xFFFFu);
    return (float)__builtin_bit_cast(_Float16, (unsigned short)h);
}
template <> MXP_DEV float u4_elem<BF16>(const uint4& v, int k) {
    const unsigned w[4] = {v.x, v.y, v.z, v.w};
    return __uint_as_float((k & 1) ? (w[k >> 1] & 0xFFFF0000u) : (w[k >> 1] << 16));
}

__device__ bool wait_flag(const unsigned* flag, unsigned target, int* err, int* s_abort) {
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned it = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            // a wait that expired anywhere ends every other wait at once
            if (++it > (1u << 24) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                atomicOr(err, 1);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        *s_abort = !ok;
    }
    __syncthreads();
    return !*s_abort;
}

// every wave waits for its stores to be acknowledged, then the flag counts
// one more strip
__device__ void signal_flag(unsigned* flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int ST, bool LOWER>
__global__ __launch_bounds__(256) void k_trsv(int64_t n, int nb, const typename Store<ST>::T* __restrict__ A,
                                              int64_t lda, int vec, const float* __restrict__ inv_all,
                                              const float* __restrict__ lsc, int64_t nstrips32,
                                              const double* __restrict__ rhs, double* __restrict__ tbuf,
                                              double* __restrict__ out, unsigned* flags, int* err) {
    typedef typename Store<ST>::T T;
    constexpr int RPL = 16 / (int)sizeof(T);   // rows per lane: one 16-byte load
    constexpr int RG = TS / RPL;               // lanes per column
    constexpr int CPI = 64 / RG;               // columns per wave and load
    static_assert(CPI >= 4, "part[][] also holds the four column groups of the diagonal apply");
    __shared__ double zs[1024];
    __shared__ double part[4][CPI][TS];
    __shared__ double w[TS];
    __shared__ int s_abort;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t S = (n + TS - 1) / TS, J = (n + nb - 1) / nb;
    const int64_t sidx = LOWER ? (int64_t)blockIdx.x : S - 1 - (int64_t)blockIdx.x;
    const int64_t j = sidx / (nb / TS);
    const int64_t r0 = sidx * TS;
    const int rows = (int)(n - r0 < TS ? n - r0 : TS);
    unsigned* cnt = flags;
    unsigned* ready = flags + J;
    auto strips_of = [&](int64_t b) -> unsigned {
        const int64_t kb = n - b * nb < nb ? n - b * nb : nb;
        return (unsigned)((kb + TS - 1) / TS);
    };
    if (tid < TS) w[tid] = (tid < rows) ? rhs[r0 + tid] : 0.0;
    const bool vload = vec && rows == TS;
    const int rg = lane % RG, cl = lane / RG;
    constexpr int PF = 16;                     // panel loads issued before the dependency's flag is awaited
    for (int64_t i = LOWER ? 0 : J - 1; i != j; i += LOWER ? 1 : -1) {
        const int64_t c0 = i * nb;
        const int kbi = (int)(n - c0 < nb ? n - c0 : nb);
        const int q = (kbi + 3) / 4, cb = wv * q, ce = (cb + q < kbi) ? cb + q : kbi;
        const T* base = A + r0 + RPL * rg + c0 * lda;
        // the factor panel does not depend on the flag: its loads overlap the
        // wait.  The loads carry no condition (a column past the range reads
        // column 0 and is weighted zero below): a load under a branch ends in
        // a wait for every load in flight, which would serialise them
        // (the ragged last strip, which takes element loads below, reads the
        // 16-byte aligned inverse array instead and ignores the values)
        uint4 pre[PF];
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            const int c = cb + cl + m * CPI;
            const void* src = vload ? (const void*)(base + (int64_t)(c < ce ? c : 0) * lda) : (const void*)inv_all;
            pre[m] = *(const uint4*)src;
        }
        if (!wait_flag(&ready[i], strips_of(i), err, &s_abort)) return;
#pragma unroll
        for (int m = 0; m < PF; ++m) pin4(pre[m]);
        for (int c = tid; c < kbi; c += 256) zs[c] = get_shared(out + c0 + c);
        __syncthreads();
        double acc[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) acc[k] = 0.0;
        if (vload) {
#pragma unroll
            for (int m = 0; m < PF; ++m) {
                const int c = cb + cl + m * CPI;
                const double zc = c < ce ? zs[c] : 0.0;
#pragma unroll
                for (int k = 0; k < RPL; ++k) acc[k] += (double)u4_elem<ST>(pre[m], k) * zc;
            }
#pragma unroll 4
            for (int c = cb + cl + PF * CPI; c < ce; c += CPI) {
                const uint4 v = *(const uint4*)(base + (int64_t)c * lda);
                const T* e = (const T*)&v;
                const double zc = zs[c];
#pragma unroll
                for (int k = 0; k < RPL; ++k) acc[k] += (double)Store<ST>::load(e, k) * zc;
            }
        } else {
            for (int c = cb + cl; c < ce; c += CPI) {
                const double zc = zs[c];
#pragma unroll
                for (int k = 0; k < RPL; ++k)
                    if (RPL * rg + k < rows) acc[k] += (double)Store<ST>::load(base, (int64_t)c * lda + k) * zc;
            }
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) part[wv][cl][RPL * rg + k] = acc[k];
        __syncthreads();
        if (tid < rows) {
            double t = 0.0;
            for (int u = 0; u < 4; ++u)
                for (int v2 = 0; v2 < CPI; ++v2) t += part[u][v2][tid];
            if (LOWER) t /= (double)lsc[i * nstrips32 + (r0 + tid) / 32];
            w[tid] -= t;
        }
    }
    // this strip's rows of the diagonal-block inverse (lower / upper
    // triangular: only the columns up to / from the strip's rows), four rows
    // per lane with 16-byte loads, the waves splitting the columns.  They do
    // not depend on the other strips: the first batch is loaded while the
    // strips of the block meet.
    const int64_t cj = j * nb;
    const int kbj = (int)(n - cj < nb ? n - cj : nb);
    const int rl0 = (int)(r0 - cj);
    const int clo = LOWER ? 0 : rl0, chi = LOWER ? (rl0 + TS < kbj ? rl0 + TS : kbj) : kbj;
    const int qv = (chi - clo + 3) / 4, cbv = clo + wv * qv, cev = (cbv + qv < chi) ? cbv + qv : chi;
    const int rsub = lane % 16, csub = lane / 16;
    const float* colbase = inv_all + j * (int64_t)nb * nb + rl0 + 4 * rsub;
    // this strip's rows of the block right-hand side are final
    if (tid < rows) put_shared(tbuf + r0 + tid, w[tid]);
    signal_flag(&cnt[j]);
    // (issued after the signal, whose wait for this wave's stores would also
    // wait for them)
    constexpr int NIV = 16;
    float4 iv0[NIV];
#pragma unroll
    for (int t = 0; t < NIV; ++t) {
        const int c = cbv + csub + 4 * t;
        iv0[t] = *(const float4*)(colbase + (int64_t)(c < cev ? c : clo) * nb);
    }
    if (!wait_flag(&cnt[j], strips_of(j), err, &s_abort)) return;
#pragma unroll
    for (int t = 0; t < NIV; ++t) pin4f(iv0[t]);
    for (int c = tid; c < kbj; c += 256) zs[c] = get_shared(tbuf + cj + c);
    __syncthreads();
    {
        const int cb = cbv, ce = cev;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        auto fma4 = [&](const float4 v, double zc) {
            acc[0] += (double)v.x * zc;
            acc[1] += (double)v.y * zc;
            acc[2] += (double)v.z * zc;
            acc[3] += (double)v.w * zc;
        };
#pragma unroll
        for (int t = 0; t < NIV; ++t) {
            const int c = cb + csub + 4 * t;
            fma4(iv0[t], c < ce ? zs[c] : 0.0);
        }
        // the rest in batches of NIV loads in flight at once, without
        // conditions (a column past the range reads column clo and is
        // weighted zero)
        for (int c0b = cb + csub + 4 * NIV; c0b < ce; c0b += 4 * NIV) {
            float4 iv[NIV];
#pragma unroll
            for (int t = 0; t < NIV; ++t) {
                const int c = c0b + 4 * t;
                iv[t] = *(const float4*)(colbase + (int64_t)(c < ce ? c : clo) * nb);
            }
#pragma unroll
            for (int t = 0; t < NIV; ++t) {
                const int c = c0b + 4 * t;
                fma4(iv[t], c < ce ? zs[c] : 0.0);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) part[wv][csub][4 * rsub + k] = acc[k];
    }
    __syncthreads();
    if (tid < rows) {
        double t = 0.0;
        for (int u = 0; u < 4; ++u)
            for (int v2 = 0; v2 < 4; ++v2) t += part[u][v2][tid];
        put_shared(out + r0 + tid, t);
    }
    signal_flag(&ready[j]);
}

__global__ void k_zero_u32(unsigned* p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = 0u;
}

static int64_t trsv_flag_words(int64_t n) { return 4 * (n / TS + 2) + 2; }

size_t prec_work_bytes(int64_t n, int nr) {
    // R (n x nr), Y, Tb (n each), flags + error word
    return (size_t)(n * nr + 2 * n) * 8 + (size_t)trsv_flag_words(n) * 4 + 256;
}

static int* prec_err_word(double* W, int64_t n, int nr) {
    return (int*)((unsigned*)(W + n * nr + 2 * n) + trsv_flag_words(n) - 2);
}

hipError_t prec_err_reset(double* W, int64_t n, int nr, hipStream_t s) {
    k_zero_u32<<<1, 256, 0, s>>>((unsigned*)prec_err_word(W, n, nr), 1);
    return hipGetLastError();
}

hipError_t prec_err_read(double* W, int64_t n, int nr, int* err, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(err, prec_err_word(W, n, nr), sizeof(int), hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    return e;
}

template <int ST>
static hipError_t prec_typed(const PrecPlan& p, const double* V, int64_t ldv, double* Z, int64_t ldz, int nr,
                             double* W, hipStream_t s) {
    typedef typename Store<ST>::T T;
    const int64_t n = p.n, nb = p.nb;
    const int64_t J = (n + nb - 1) / nb;
    const int64_t nstrips32 = (n + 31) / 32;
    const int64_t S = (n + TS - 1) / TS;
    double* R = W;                 // S V, nr columns
    double* Y = W + n * nr;        // forward solution
    double* Tb = Y + n;            // block right-hand sides
    unsigned* flags = (unsigned*)(Tb + n);
    int* err = prec_err_word(W, n, nr);
    const int vec = ((p.lda * (int64_t)sizeof(T)) % 16 == 0 && ((uintptr_t)p.A) % 16 == 0) ? 1 : 0;
    hipEvent_t pt = prof::begin(prof::PREC, s);
    k_scale_rows<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, p.rowscale, V, ldv, R, nr);
    for (int r = 0; r < nr; ++r) {
        k_zero_u32<<<(unsigned)((4 * J + 255) / 256), 256, 0, s>>>(flags, 4 * J);
        k_trsv<ST, true><<<(unsigned)S, 256, 0, s>>>(n, (int)nb, (const T*)p.A, p.lda, vec, p.linv_full, p.lsc,
                                                     nstrips32, R + r * n, Tb, Y, flags, err);
        k_trsv<ST, false><<<(unsigned)S, 256, 0, s>>>(n, (int)nb, (const T*)p.A, p.lda, vec, p.uinv_full, nullptr,
                                                      nstrips32, Y, Tb, Z + r * ldz, flags + 2 * J, err);
    }
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
