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
// One kernel per triangular solve, every right-hand side at once (each
// right-hand side with its own flags).  Work-group = one strip of TS rows;
// strips are processed as a dataflow: a strip of block j accumulates the
// products of its rows of the off-diagonal factor with every dependency
// block's solution as soon as that block is published (flag `ready`),
// publishes its rows of the block right-hand side (its strip flag), and
// applies its rows of the FP32 inverse of the diagonal block once the strips
// those rows depend on have published theirs (the inverse is triangular:
// the strips above it in the block for L, below it for U); it then counts
// itself into the block's `ready`.  Forward (L): dependencies are the blocks
// before j, strips run in increasing order; backward (U): the blocks after
// j, strips in decreasing order.
//
// A work-group takes its position (right-hand side, strip) from a counter
// of the launch when it starts, not from its index, and every wait is on
// strips of earlier positions, so every wait is on work-groups that have
// started: the earliest unfinished one waits on none and runs to its end.
// The launch then always drains, whatever else holds the device: the
// hardware deals the indices out to the XCDs, each dispatching its share in
// order, and with other launches on other streams it can hold back a
// launch's remaining work-groups while that launch's resident ones spin.
// Each wait is still bounded and on expiry sets *err and lets the
// work-group exit.  All sums are taken in a fixed order (deterministic
// results).
#ifndef MXP_TRSV_TS
#define MXP_TRSV_TS 64
#endif
constexpr int TS = MXP_TRSV_TS;

// Values exchanged between work-groups (block solutions, block right-hand
// sides) are written and read with device-scope atomic accesses, which go to
// the device's coherence point instead of an XCD's L2.  A flag is raised
// after every wave's stores are released (sync_release) and a work-group
// barrier; a waiter that sees the flag reads after it (sync_acquire, then
// the barrier that lets its other threads read); see common.hpp.
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
        if (ok) sync_acquire();
        *s_abort = !ok;
    }
    __syncthreads();
    return !*s_abort;
}

// bounded wait, by the first wave, until the cnt flags f[0 .. cnt) are all
// raised (cnt <= 64: one lane per flag)
__device__ bool wait_all(const unsigned* f, int cnt, int* err, int* s_abort) {
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        int ok = 1;
        unsigned it = 0;
        for (;;) {
            const bool up = l >= cnt || __hip_atomic_load(f + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            if (__all(up)) break;
            if (++it > (1u << 24) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                if (l == 0) atomicOr(err, 1);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (ok) sync_acquire();
        if (l == 0) *s_abort = !ok;
    }
    __syncthreads();
    return !*s_abort;
}

// every wave's stores are released at agent scope and precede the barrier;
// the flag then counts one more strip with release semantics
__device__ void signal_flag(unsigned* flag) {
    sync_release();
    __syncthreads();
    if (threadIdx.x == 0) {
        sync_release();
        __hip_atomic_fetch_add(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int ST, bool LOWER>
__global__ __launch_bounds__(256) void k_trsv(int64_t n, int nb, int db, const typename Store<ST>::T* __restrict__ A,
                                              int64_t lda, int vec, const float* __restrict__ inv_all,
                                              const float* __restrict__ lsc, int64_t nstrips32,
                                              const double* __restrict__ rhs, int64_t ld_rhs,
                                              double* __restrict__ tbuf, double* __restrict__ out, int64_t ld_out,
                                              unsigned* flags, int64_t flag_stride, unsigned* ticket,
                                              int* err) {
    typedef typename Store<ST>::T T;
    constexpr int RPL = 16 / (int)sizeof(T);   // rows per lane: one 16-byte load
    constexpr int RG = TS / RPL;               // lanes per column
    constexpr int CPI = 64 / RG;               // columns per wave and load
    __shared__ double zs[1024];
    constexpr int PCOLS = CPI > 64 / (TS / 8) ? CPI : 64 / (TS / 8);   // column groups: panels, diagonal apply
    __shared__ double part[4][PCOLS][TS];
    __shared__ double w[TS];
    __shared__ int s_abort;
    __shared__ unsigned s_pos;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // position in start order: strip pos % S of right-hand side pos / S (the
    // grid is S x nrhs work-groups)
    if (tid == 0) s_pos = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t S = (n + TS - 1) / TS, J = (n + nb - 1) / nb, gb = db / nb;
    const int64_t pos = s_pos, px = pos % S, py = pos / S;
    // right-hand side py: its own vectors, block buffer and flags
    rhs += py * ld_rhs;
    out += py * ld_out;
    tbuf += py * n;
    flags += py * flag_stride;
    // the substitution's diagonal blocks (size db, a multiple of nb: gb factor
    // blocks each) are the dataflow's steps; the off-diagonal products go by
    // factor block (each with its own strip factors)
    const int64_t sidx = LOWER ? px : S - 1 - px;
    const int64_t j = sidx / (db / TS);
    const int64_t first = j * gb, last = (first + gb < J ? first + gb : J) - 1;
    const int64_t r0 = sidx * TS;
    const int rows = (int)(n - r0 < TS ? n - r0 : TS);
    unsigned* sflag = flags;          // one per strip: its rows of the block right-hand side are published
    unsigned* ready = flags + S;      // one per block: strips that have published their solution rows
    auto strips_of = [&](int64_t b) -> unsigned {
        const int64_t kb = n - b * db < db ? n - b * db : db;
        return (unsigned)((kb + TS - 1) / TS);
    };
    if (tid < TS) w[tid] = (tid < rows) ? rhs[r0 + tid] : 0.0;
    const bool vload = vec && rows == TS;
    const int rg = lane % RG, cl = lane / RG;
    constexpr int PF = 16;                     // panel loads issued before the dependency's flag is awaited
    // The factor panels do not depend on the flags: the panel of the next
    // dependency block is loaded while the current one is awaited and applied
    // (two buffers, the loop taken two blocks at a time).  The loads carry no
    // condition (a column past the range reads column 0 and is weighted zero
    // below): a load under a branch ends in a wait for every load in flight,
    // which would serialise them (the ragged last strip, which takes element
    // loads below, reads the 16-byte aligned inverse array instead and
    // ignores the values).
    const int64_t istep = LOWER ? 1 : -1;
    auto in_range = [&](int64_t i) { return LOWER ? (i < first) : (i > last); };
    auto issue = [&](int64_t i, uint4* dst) {
        const int64_t c0 = i * nb;
        const int kbi = (int)(n - c0 < nb ? n - c0 : nb);
        const int q = (kbi + 3) / 4, cb = wv * q, ce = (cb + q < kbi) ? cb + q : kbi;
        const T* base = A + r0 + RPL * rg + c0 * lda;
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            const int c = cb + cl + m * CPI;
            const void* src = vload ? (const void*)(base + (int64_t)(c < ce ? c : 0) * lda) : (const void*)inv_all;
            dst[m] = *(const uint4*)src;
        }
    };
    // one dependency block: wait for it, multiply its panel (prefetched in
    // pre) with its solution and subtract from w
    auto dep = [&](int64_t i, uint4* pre, uint4* nxt) -> bool {
        const int64_t c0 = i * nb;
        const int kbi = (int)(n - c0 < nb ? n - c0 : nb);
        const int q = (kbi + 3) / 4, cb = wv * q, ce = (cb + q < kbi) ? cb + q : kbi;
        const T* base = A + r0 + RPL * rg + c0 * lda;
        if (in_range(i + istep)) issue(i + istep, nxt);
        if (!wait_flag(&ready[i / gb], strips_of(i / gb), err, &s_abort)) return false;
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
        return true;
    };
    {
        uint4 pa[PF], pb[PF];
        int64_t i = LOWER ? 0 : J - 1;
        if (in_range(i)) issue(i, pa);
        for (;;) {
            if (!in_range(i)) break;
            if (!dep(i, pa, pb)) return;
            i += istep;
            if (!in_range(i)) break;
            if (!dep(i, pb, pa)) return;
            i += istep;
        }
    }
    // The strip's rows of its diagonal-block inverse (lower / upper
    // triangular: a row takes the columns up to / from itself), applied in two
    // half strips of HS rows.  A lane: four consecutive rows (16-byte loads),
    // one of CS column groups; the waves split a half strip's columns.  The
    // first batch of loads is issued while the strips it depends on publish.
    const int64_t cj = j * db;
    const int kbj = (int)(n - cj < db ? n - cj : db);
    const int nst = (int)strips_of(j);
    const int s_in = (int)((r0 - cj) / TS);
    constexpr int HS = TS / 2, RQ = HS / 4, CS = 64 / RQ;
    static_assert(PCOLS >= CS, "part[][] also holds the column groups of the diagonal apply");
    const int rsub = lane % RQ, csub = lane / RQ;
    const float* blkinv = inv_all + j * (int64_t)db * db + 4 * rsub;
    struct Half {
        int r0, rows, clo, cb, ce;
    };
    auto half = [&](int h) {
        Half H;
        H.r0 = HS * h;
        H.rows = kbj - H.r0 < HS ? kbj - H.r0 : HS;               // <= 0: nothing to do
        H.clo = LOWER ? 0 : H.r0;
        const int chi = LOWER ? (H.r0 + HS < kbj ? H.r0 + HS : kbj) : kbj;
        const int q = chi > H.clo ? (chi - H.clo + 3) / 4 : 0;
        H.cb = H.clo + wv * q;
        H.ce = H.cb + q < chi ? H.cb + q : chi;
        return H;
    };
    const Half HA = half(2 * s_in), HB = half(2 * s_in + 1);
    // this strip's rows of the block right-hand side are final
    if (tid < rows) put_shared(tbuf + r0 + tid, w[tid]);
    signal_flag(&sflag[sidx]);
    // (issued after the signal, whose wait for this wave's stores would also
    // wait for them)
#ifndef MXP_TRSV_NIV
#define MXP_TRSV_NIV 16
#endif
    constexpr int NIV = MXP_TRSV_NIV;     // inverse loads in flight per lane (16 bytes each)
    float4 iv0[NIV];
    {
        const float* rb = blkinv + HA.r0;
#pragma unroll
        for (int t = 0; t < NIV; ++t) {
            const int c = HA.cb + csub + CS * t;
            iv0[t] = *(const float4*)(rb + (int64_t)(c < HA.ce ? c : HA.clo) * db);
        }
    }
    // the strips whose right-hand side rows this strip's rows take: those
    // above it in the block (L), below it (U)
    const int64_t sb = sidx - s_in;
    if (!(LOWER ? wait_all(sflag + sb, s_in, err, &s_abort)
                : wait_all(sflag + sidx + 1, nst - 1 - s_in, err, &s_abort)))
        return;
#pragma unroll
    for (int t = 0; t < NIV; ++t) pin4f(iv0[t]);
    {
        const int zlo = LOWER ? 0 : s_in * TS, zhi = LOWER ? s_in * TS + rows : kbj;
        for (int c = zlo + tid; c < zhi; c += 256) zs[c] = get_shared(tbuf + cj + c);
    }
    __syncthreads();
    // one half strip: its columns in batches of NIV loads in flight at once,
    // without conditions (a column past the range reads column clo and is
    // weighted zero); the first batch is given (pre) or loaded here
    auto apply = [&](const Half& H, float4 (&pre)[NIV], bool has_pre) {
        const float* rb = blkinv + H.r0;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        auto fma4 = [&](const float4 v, double zc) {
            acc[0] += (double)v.x * zc;
            acc[1] += (double)v.y * zc;
            acc[2] += (double)v.z * zc;
            acc[3] += (double)v.w * zc;
        };
        int c0b = H.cb + csub;
        if (has_pre) {
#pragma unroll
            for (int t = 0; t < NIV; ++t) {
                const int c = c0b + CS * t;
                fma4(pre[t], c < H.ce ? zs[c] : 0.0);
            }
            c0b += CS * NIV;
        }
        for (; c0b < H.ce; c0b += CS * NIV) {
            float4 iv[NIV];
#pragma unroll
            for (int t = 0; t < NIV; ++t) {
                const int c = c0b + CS * t;
                iv[t] = *(const float4*)(rb + (int64_t)(c < H.ce ? c : H.clo) * db);
            }
#pragma unroll
            for (int t = 0; t < NIV; ++t) {
                const int c = c0b + CS * t;
                fma4(iv[t], c < H.ce ? zs[c] : 0.0);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) part[wv][csub][4 * rsub + k] = acc[k];
        __syncthreads();
        if (tid < H.rows) {
            double t = 0.0;
            for (int u = 0; u < 4; ++u)
                for (int v2 = 0; v2 < CS; ++v2) t += part[u][v2][tid];
            put_shared(out + cj + H.r0 + tid, t);
        }
        __syncthreads();                      // part[] free for the next half
    };
    if (HA.rows > 0) apply(HA, iv0, true);
    if (HB.rows > 0) apply(HB, iv0, false);
    signal_flag(&ready[j]);
}

__global__ void k_zero_u32(unsigned* p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// flag words of one right-hand side: the strip flags (S = ceil(n / TS)) and
// block flags (J = ceil(n / nb), nb >= 64) of both solves; those of the
// first right-hand side also hold the two solves' start-order counters
// (words 2 (S + J) and 2 (S + J) + 1)
static int64_t trsv_flag_words(int64_t n) {
    constexpr int64_t u = TS < 64 ? TS : 64;
    return 4 * (n / u + 2);
}

size_t prec_work_bytes(int64_t n, int nr) {
    // S V, forward solution, block right-hand sides (n x nr each), flags, error word
    return (size_t)(3 * n * nr) * 8 + (size_t)(trsv_flag_words(n) * nr) * 4 + 256;
}

static int* prec_err_word(double* W, int64_t n, int nr) {
    return (int*)((unsigned*)(W + 3 * n * nr) + trsv_flag_words(n) * nr);
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
    double* R = W;                 // S V, nr columns (ld n)
    double* Y = W + n * nr;        // forward solutions
    double* Tb = Y + n * nr;       // block right-hand sides
    unsigned* flags = (unsigned*)(Tb + n * nr);
    const int64_t fw = trsv_flag_words(n);
    int* err = prec_err_word(W, n, nr);
    const int vec = ((p.lda * (int64_t)sizeof(T)) % 16 == 0 && ((uintptr_t)p.A) % 16 == 0) ? 1 : 0;
    hipEvent_t pt = prof::begin(prof::PREC, s);
    k_scale_rows<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, p.rowscale, V, ldv, R, nr);
    k_zero_u32<<<(unsigned)((fw * nr + 255) / 256), 256, 0, s>>>(flags, fw * nr);
    const int db = (int)prec_block(nb);
    k_trsv<ST, true><<<dim3((unsigned)S, (unsigned)nr), 256, 0, s>>>(n, (int)nb, db, (const T*)p.A, p.lda, vec,
                                                                     p.linv_full, p.lsc, nstrips32, R, n, Tb, Y, n,
                                                                     flags, fw, flags + 2 * (S + J), err);
    k_trsv<ST, false><<<dim3((unsigned)S, (unsigned)nr), 256, 0, s>>>(n, (int)nb, db, (const T*)p.A, p.lda, vec,
                                                                      p.uinv_full, nullptr, nstrips32, Y, n, Tb, Z,
                                                                      ldz, flags + S + J, fw, flags + 2 * (S + J) + 1,
                                                                      err);
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

// ================================================================ GMRES vector kernels
// Every right-hand side runs its own GMRES in lockstep with the others:
// blockIdx.y (or the thread index of the scalar kernels) is the right-hand
// side r, and act[r] says whether r takes part in the current step (the
// others' blocks return at once).  Every reduction gives block b the fixed
// index range [b*chunk, (b+1)*chunk) and sums it in a fixed order, so
// results are identical from run to run.
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

// part[r][b] = sum over block b's range of x_r . y_r
__global__ __launch_bounds__(256) void k_dot_part(int64_t n, int64_t chunk, const double* __restrict__ x, int64_t ldx,
                                                  const double* __restrict__ y, int64_t ldy, double* __restrict__ part,
                                                  const int* __restrict__ act) {
    __shared__ double red[4];
    const int r = blockIdx.y;
    if (!act[r]) return;
    x += r * ldx;
    y += r * ldy;
    const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    double v = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) v += x[i] * y[i];
    v = block_sum(v, red);
    if (threadIdx.x == 0) part[r * 256 + blockIdx.x] = v;
}

// MGS step j of column k: h_jk = sum(part_in); w -= h_jk v_j over the
// block's range; then the partial dot for the next vector (v_{j+1} . w, or
// w . w after the last one).  V: basis vectors v_{r,j} at V + (j nr + r) n.
__global__ __launch_bounds__(256) void k_mgs(int64_t n, int64_t chunk, int nr, const double* __restrict__ V, int j,
                                             int last, double* __restrict__ W, const double* __restrict__ part_in,
                                             double* __restrict__ part_out, double* __restrict__ H, int ldh, int k,
                                             const int* __restrict__ act) {
    __shared__ double red[4];
    const int r = blockIdx.y;
    if (!act[r]) return;
    const double* vj = V + ((int64_t)j * nr + r) * n;
    const double* vnext = last ? nullptr : V + ((int64_t)(j + 1) * nr + r) * n;
    double* w = W + (int64_t)r * n;
    const double h = sum_parts(part_in + r * 256, gridDim.x, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) H[(int64_t)r * ldh * (ldh - 1) + j + (int64_t)k * ldh] = h;
    const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    double v = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double wi = w[i] - h * vj[i];
        w[i] = wi;
        v += (vnext ? vnext[i] : wi) * wi;
    }
    v = block_sum(v, red);
    if (threadIdx.x == 0) part_out[r * 256 + blockIdx.x] = v;
}

// h = sqrt(sum(part)); H[k+1][k] = h; v_{k+1} = w / h (0 on exact breakdown)
__global__ __launch_bounds__(256) void k_normalize(int64_t n, int64_t chunk, int nr, const double* __restrict__ part,
                                                   const double* __restrict__ W, double* __restrict__ V, int k,
                                                   double* __restrict__ H, int ldh, const int* __restrict__ act) {
    __shared__ double red[4];
    const int r = blockIdx.y;
    if (!act[r]) return;
    const double h = sqrt(sum_parts(part + r * 256, gridDim.x, red));
    if (blockIdx.x == 0 && threadIdx.x == 0) H[(int64_t)r * ldh * (ldh - 1) + (k + 1) + (int64_t)k * ldh] = h;
    const double* w = W + (int64_t)r * n;
    double* v = V + ((int64_t)(k + 1) * nr + r) * n;
    const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) v[i] = (h > 0.0) ? w[i] / h : 0.0;
}

// out[r] = sqrt(sum(part[r]))
__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ part, int nparts, double* out,
                                                    int out_stride, const int* __restrict__ act) {
    __shared__ double red[4];
    const int r = blockIdx.x;
    if (!act[r]) return;
    const double v = sum_parts(part + r * 256, nparts, red);
    if (threadIdx.x == 0) out[r * out_stride] = sqrt(v);
}

// v_{r,0} = z_r / beta_r; g_r = beta_r e_1
__global__ __launch_bounds__(256) void k_start_basis(int64_t n, const double* __restrict__ Z, const double* sc,
                                                     int sc_stride, double* __restrict__ V, int nr,
                                                     double* __restrict__ g, int ldg, const int* __restrict__ act) {
    const int r = blockIdx.y;
    if (!act[r]) return;
    const double b = sc[r * sc_stride];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < ldg) g[r * ldg + threadIdx.x] = threadIdx.x == 0 ? b : 0.0;
    if (i < n) V[(int64_t)r * n + i] = (b > 0.0) ? Z[(int64_t)r * n + i] / b : 0.0;
}

// Column k of each active H_r (column-major, ldh = m + 1): apply rotations
// 0..k-1, form rotation k that zeroes H[k+1][k], rotate g.  flag[r] = 1 when
// |g[k+1]| <= tau ||x_r|| or H[k+1][k] was 0 (exact breakdown).
__global__ void k_givens(int nr, int k, double* H, int ldh, double* cs, double* sn, double* g,
                         const double* sc, int sc_stride, double tau, int* flag, const int* __restrict__ act) {
    const int r = threadIdx.x;
    if (r >= nr || !act[r]) return;
    double* h = H + (int64_t)r * ldh * (ldh - 1) + (int64_t)k * ldh;
    double* c_ = cs + r * ldh;
    double* s_ = sn + r * ldh;
    double* gr = g + r * ldh;
    const double hsub = h[k + 1];
    for (int i = 0; i < k; ++i) {
        const double a = h[i], b = h[i + 1];
        h[i] = c_[i] * a + s_[i] * b;
        h[i + 1] = -s_[i] * a + c_[i] * b;
    }
    const double a = h[k], b = h[k + 1];
    const double rho = hypot(a, b);
    const double c = (rho > 0.0) ? a / rho : 1.0, s = (rho > 0.0) ? b / rho : 0.0;
    c_[k] = c;
    s_[k] = s;
    h[k] = rho;
    h[k + 1] = 0.0;
    const double gk = gr[k];
    gr[k + 1] = -s * gk;
    gr[k] = c * gk;
    const double xnorm = sc[r * sc_stride];
    flag[r] = (fabs(gr[k + 1]) <= tau * xnorm || hsub == 0.0) ? 1 : 0;
}

// y_r = R_r^-1 g_r (R_r = rotated H_r[0:k_r, 0:k_r]), k_r = kdim[r]
__global__ void k_backsub(int nr, const double* H, int ldh, const double* g, double* y, const int* kdim) {
    const int r = threadIdx.x;
    if (r >= nr) return;
    const int k = kdim[r];
    const double* Hr = H + (int64_t)r * ldh * (ldh - 1);
    const double* gr = g + r * ldh;
    double* yr = y + r * ldh;
    for (int i = k - 1; i >= 0; --i) {
        double t = gr[i];
        for (int l = i + 1; l < k; ++l) t -= Hr[i + (int64_t)l * ldh] * yr[l];
        yr[i] = t / Hr[i + (int64_t)i * ldh];
    }
}

// x_r += V_r[:, 0:k_r] y_r
__global__ __launch_bounds__(256) void k_axpy_basis(int64_t n, int nr, const double* __restrict__ V,
                                                    const double* __restrict__ y, int ldy, const int* kdim,
                                                    double* __restrict__ X, int64_t ldx) {
    const int r = blockIdx.y;
    const int k = kdim[r];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n || k == 0) return;
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += y[r * ldy + j] * V[((int64_t)j * nr + r) * n + i];
    X[r * ldx + i] += acc;
}

__global__ void k_set_i32(int* p, int n, const int* src) {
    const int i = threadIdx.x;
    if (i < n) p[i] = src ? src[i] : 0;
}

// ---- host wrappers (all right-hand sides at once; V is (m + 1) x nr x n)
hipError_t gm_norms(int64_t n, int nr, const double* X, int64_t ldx, double* out, int out_stride, double* part,
                    const int* act, hipStream_t s) {
    const int nbk = red_blocks(n);
    const int64_t chunk = (n + nbk - 1) / nbk;
    k_dot_part<<<dim3(nbk, nr), 256, 0, s>>>(n, chunk, X, ldx, X, ldx, part, act);
    k_norm_final<<<nr, 256, 0, s>>>(part, nbk, out, out_stride, act);
    return hipGetLastError();
}

hipError_t gm_start(int64_t n, int nr, const double* Z, const double* sc, int sc_stride, double* V, double* g,
                    int ldg, const int* act, hipStream_t s) {
    k_start_basis<<<dim3((unsigned)((n + 255) / 256), nr), 256, 0, s>>>(n, Z, sc, sc_stride, V, nr, g, ldg, act);
    return hipGetLastError();
}

hipError_t gm_arnoldi(int64_t n, int nr, double* V, int k, double* W, double* part, double* H, int ldh,
                      const int* act, hipStream_t s) {
    const int nbk = red_blocks(n);
    const int64_t chunk = (n + nbk - 1) / nbk;
    k_dot_part<<<dim3(nbk, nr), 256, 0, s>>>(n, chunk, V, n, W, n, part, act);
    for (int j = 0; j <= k; ++j) {
        const double* pin = part + (j & 1) * 256 * nr;
        double* pout = part + ((j + 1) & 1) * 256 * nr;
        k_mgs<<<dim3(nbk, nr), 256, 0, s>>>(n, chunk, nr, V, j, j == k, W, pin, pout, H, ldh, k, act);
    }
    k_normalize<<<dim3(nbk, nr), 256, 0, s>>>(n, chunk, nr, part + ((k + 1) & 1) * 256 * nr, W, V, k, H, ldh, act);
    return hipGetLastError();
}

hipError_t gm_givens(int nr, int k, double* H, int ldh, double* cs, double* sn, double* g, const double* sc,
                     int sc_stride, double tau, int* flag, const int* act, hipStream_t s) {
    k_givens<<<1, 64, 0, s>>>(nr, k, H, ldh, cs, sn, g, sc, sc_stride, tau, flag, act);
    return hipGetLastError();
}

hipError_t gm_update(int64_t n, int nr, const double* H, int ldh, const double* g, double* y, const int* kdim,
                     const double* V, double* X, int64_t ldx, hipStream_t s) {
    k_backsub<<<1, 64, 0, s>>>(nr, H, ldh, g, y, kdim);
    k_axpy_basis<<<dim3((unsigned)((n + 255) / 256), nr), 256, 0, s>>>(n, nr, V, y, ldh, kdim, X, ldx);
    return hipGetLastError();
}

hipError_t set_i32(int* dst, int n, const int* src_dev, hipStream_t s) {
    k_set_i32<<<1, 64, 0, s>>>(dst, n, src_dev);
    return hipGetLastError();
}

}  // namespace mxp
