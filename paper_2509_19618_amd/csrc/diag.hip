// diag.hip -- FP32 LU without pivoting of one diagonal block (the panel
// factorisation of the right-looking blocked LU; paper: "Algorithmic
// Framework" and its Figure 1: the panel is factored in 32-bit arithmetic
// before the 16-bit trailing update).
//
// The block is at most 1024 x 1024 and its factorisation is a chain of small
// dependent steps over 32 x 32 tiles of an FP32 copy T (column-major, ld =
// ldt), right-looking:
//
//   for t = 0 .. P-1   (P = kbp / 32)
//     phase L(t): the leader (wave 0 of work-group 0) applies the last
//                 update to tile (t,t) and factors it in registers (row r of
//                 the tile in lane r); every other wave applies update t-1
//                 to the other trailing tiles;
//     phase T(t): tiles (i,t) <- tile(i,t) U_tt^-1 and (t,j) <- L_tt^-1 tile(t,j),
//                 each by substitution against the factored tile (t,t)
//   (the first access to a tile reads it from A; T holds it from then on)
//   phase inv:   the inverses of the 32 x 32 unit-lower and upper diagonal
//                tiles (one wave each, all at once);
//   phase asm:   off-diagonal blocks of the 64 x 64 sub-block inverses.
//
// The chain of dependent steps is the leaf factorisations and the
// substitutions; the tile inverses, needed only by the strip TRSMs that
// follow, stay off it.
//
// One launch of a few work-groups of four waves (each fits on a CU beside a
// work-group of the concurrent trailing update).  Every wave works on its
// own: it claims tasks of the current phase from a device-wide counter,
// counts them done, and the wave that completes a phase opens the next one.
// Work-groups that start late simply join the current phase, so the leader
// never waits for a helper to be scheduled.  T and the tile inverses are
// read and written with device-scope accesses (they go to the device's
// coherence point).  A wave counts a task done after a release of its stores
// to T (sync_release: the wave's stores acknowledged), the wave that closes
// a phase opens the next one the same way, and a wave that sees a phase open
// reads after it (sync_acquire; see common.hpp for why the hardware form of
// these needs no cache maintenance).  The final copies to A and Trm, read
// only after the launch, are written after the completion.  Every wait is
// bounded: on expiry it records an error in *info and the wave exits.
//
// Every 32 x 32 x 32 product is one wave's chain of sixteen
// v_mfma_f32_32x32x2f32; a substitution is one wave's chain of FMAs with
// the triangular factor read from LDS four entries at a time.  The kernel also writes the inverses of the 64 x 64
// unit-lower (column-major) and upper (row-major) diagonal sub-blocks used by
// the strip TRSMs, the factored block back into A in the storage format, and
// a row-major copy Trm of T.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace mxp {

namespace {

typedef float f16v_t __attribute__((ext_vector_type(16)));
typedef float v32f __attribute__((ext_vector_type(32)));

// four waves (one per SIMD, at most 256 registers each, 34 KB of LDS): a
// work-group then fits on a CU beside one work-group of the concurrent
// trailing update instead of waiting for a whole CU to drain
constexpr int DW = 4;              // waves of the work-group
constexpr int DT = DW * 64;        // threads
constexpr int TP = 33;             // LDS pitch of a staged 32 x 32 tile (column-major)
constexpr int SP = 36;             // LDS pitch of a staged triangular factor (16-byte rows)
constexpr int TILE_F = 32 * SP;    // floats of one staging buffer

// v, hidden from the optimiser (keeps loop-invariant per-lane constants
// from being hoisted out of the block loop and held in registers throughout)
MXP_DEV int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// LDS accesses of one wave execute in order; this keeps the compiler from
// moving them across each other (reads through float4 and writes through
// float do not alias by type)
MXP_DEV void lds_order() { asm volatile("" ::: "memory"); }

// v, computed before this point in program order (the instruction selector
// otherwise sinks arithmetic of an unrolled chain away from its loads)
MXP_DEV void pin(float& v) { asm volatile("" : "+v"(v)); }

MXP_DEV float rl(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }

// device-scope accesses of data shared between work-groups
MXP_DEV float gld(const float* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MXP_DEV void gst(float* p, float v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
MXP_DEV int ild(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// s[c*TP + r] = g[r + c*ld] for r, c < 32 (lanes along r: coalesced)
MXP_DEV void stage_cm(float* s, const float* g, int64_t ld, int r, int h) {
    float v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = gld(g + (int64_t)(2 * q) * ld + (r + h * (int)ld));
#pragma unroll
    for (int q = 0; q < 16; ++q) s[(2 * q + h) * TP + r] = v[q];
}

// s[c*TP + r] = g[r*ld + c] for r, c < 32 (lanes along c: coalesced)
MXP_DEV void stage_rm(float* s, const float* g, int64_t ld, int c, int h) {
    float v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = gld(g + (int64_t)(2 * q) * ld + (c + h * (int)ld));
#pragma unroll
    for (int q = 0; q < 16; ++q) s[c * TP + 2 * q + h] = v[q];
}

// Product R = P Q of two 32 x 32 operands.  On return register q of lane l
// holds R[l % 32][cc(q, l)], cc = 8(q/4) + 4(l/32) + q%4: the MFMA computes
// R^T = Q^T P^T, so that a result column is spread over 32 consecutive lanes
// and is written with one coalesced access.  With r = l % 32 and
// k = 2 k2 + l / 32, fp(k2) = P[r][k] and fq(k2) = Q[k][r]; the fetchers
// split their addresses into a uniform part (depending on k2 only) and one
// 32-bit lane offset, which keeps the sixteen loads in two registers.
template <class FP, class FQ>
MXP_DEV f16v_t prod32(FP fp, FQ fq) {
    float a[16], b[16];
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) {
        b[k2] = fq(k2);
        a[k2] = fp(k2);
    }
    f16v_t acc = {};
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b[k2], a[k2], acc, 0, 0, 0);
    return acc;
}

MXP_DEV int res_col(int q, int lh) { return 8 * (q >> 2) + 4 * lh + (q & 3); }
// uniform part of res_col
MXP_DEV int res_colu(int q) { return 8 * (q >> 2) + (q & 3); }

// phases of one diagonal-block LU and their sizes (see the file comment):
// 2t L(t), 2t + 1 T(t), 2P inv, 2P + 1 asm
constexpr int NPMAX = 2 * 32 + 2;   // phases for kbp <= 1024
MXP_DEV int phase_claims(int ph, int P) {
    if (ph == 2 * P) return 2 * P;                     // tile inverses
    if (ph == 2 * P + 1) return P;                     // inverse assembly
    const int t = ph / 2;
    if (ph % 2 == 0) return t > 0 ? (P - t) * (P - t) - 1 : 0;   // L(t): updates of step t-1
    return 2 * (P - 1 - t);                            // T(t)
}
MXP_DEV bool is_lphase(int ph, int P) { return ph < 2 * P && ph % 2 == 0; }
// completions that close a phase: its claims, plus the leaf in L(t)
MXP_DEV int phase_target(int ph, int P) { return phase_claims(ph, P) + (is_lphase(ph, P) ? 1 : 0); }

}  // namespace

struct DiagOne {
    void* A;
    int64_t lda, k;
    int kb, kbp, ldt, wgs;
    float *T, *Trm, *linv, *uinv;
    int* sync;
    unsigned long long* info;
};
struct DiagGroup {
    DiagOne g[GEMM_GROUP_MAX];
    int count;
};

// One launch factors the diagonal blocks of a group of factorisations (one
// per request of the solve server, or a single one): blockIdx.y picks the
// block, each with its own phase counters; work-groups beyond a block's
// count leave at once.
template <int ST>
__global__ __launch_bounds__(DT, 2) void k_diag_lu(const DiagGroup grp) {
    extern __shared__ __attribute__((aligned(16))) float dsm[];
    const DiagOne& G = grp.g[blockIdx.y];
    if ((int)blockIdx.x >= G.wgs) return;
    typename Store<ST>::T* A = (typename Store<ST>::T*)G.A;
    const int64_t lda = G.lda, k = G.k;
    const int kb = G.kb, kbp = G.kbp, ldt = G.ldt;
    float* __restrict__ T = G.T;
    float* __restrict__ Trm = G.Trm;
    float* __restrict__ linv = G.linv;
    float* __restrict__ uinv = G.uinv;
    int* sync = G.sync;
    unsigned long long* info = G.info;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // lane-derived values, remade through opaque() before every task (see
    // refresh below)
    int lr = lane & 31, lh = lane >> 5;
    float* sA = dsm + (2 * wave) * TILE_F;       // two staging tiles per wave
    float* sB = sA + TILE_F;
    const int P = kbp / 32;
    const int NP = 2 * P + 2;
    int* phase = sync;                           // the open phase (NP = finished)
    int* claims = sync + 1;
    int* dones = sync + 1 + NPMAX;
    const bool leader = blockIdx.x == 0 && wave == 0;
    auto Tt = [&](int I, int J) -> float* { return T + 32 * I + (int64_t)(32 * J) * ldt; };
    int offA = lr + lh * ldt;                // lane offset of operand element (lr, 2 k2 + lh) of a T tile
    int offC = lr + 4 * lh * ldt;            // lane offset of result element (lr, res_col(q))
    // every task and leaf starts from fresh lane values: addresses derived
    // from them then cannot be hoisted out of the phase loop, where the
    // invariants of all task kinds would stay live at once
    auto refresh = [&]() {
        lr = opaque(lane & 31);
        lh = opaque(lane >> 5);
        offA = lr + lh * (int)ldt;
        offC = lr + 4 * lh * (int)ldt;
    };
    // operand fetchers: P[lr][k] of a T tile, P and Q of a staged LDS tile
    auto gP = [&](const float* G) { return [=](int k2) { return gld(G + (int64_t)(2 * k2) * ldt + offA); }; };
    auto sQ = [&](const float* S) { return [=](int k2) { return S[lr * TP + 2 * k2 + lh]; }; };
    auto sP = [&](const float* S) { return [=](int k2) { return S[(2 * k2 + lh) * TP + lr]; }; };
    auto Cp = [&](float* G, int q) -> float* { return G + (int64_t)res_colu(q) * ldt + offC; };
    // a final tile (I,J), held column-major in the LDS buffer S: to A in the
    // storage format and, transposed, to Trm (both with coalesced stores)
    auto store_final = [&](int I, int J, const float* S) {
        const int i = 32 * I + lr;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = 32 * J + 2 * q + lh;
            if (i < kb && j < kb) A[(k + i) + (k + j) * lda] = Store<ST>::from_f32(S[(2 * q + lh) * TP + lr]);
            Trm[(32 * J + lr) + (int64_t)(32 * I + 2 * q + lh) * ldt] = S[lr * TP + 2 * q + lh];
        }
    };
    // element (i,j) of the diagonal block in FP32 from A, padded with the
    // identity beyond kb (the first access to a tile; plain loads: A is not
    // written before that)
    auto a_el = [&](int i, int j) -> float {
        const bool in = i < kb && j < kb;
        const float v = Store<ST>::load(A, in ? (k + i) + (k + j) * lda : k + k * lda);
        return in ? v : ((i == j) ? 1.0f : 0.0f);
    };
    auto fail = [&]() {
        if (lane == 0) atomicMin(info, 1ull << 62);
    };
    // bounded wait until the open phase is at least ph (polled with relaxed
    // loads), then an acquire: the stores of the phases before ph are visible
    auto wait_phase = [&](int ph) -> bool {
        unsigned it = 0;
        while (ild(phase) < ph) {
            if (++it > (1u << 26)) {
                fail();
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        sync_acquire();
        return true;
    };
    // one more completion of ph, released by every lane (each lane counts
    // itself: one atomic of +64 per wave after the compiler combines the
    // lanes, so a phase closes at 64 completions per task); the wave that
    // closes the phase acquires the others' completions and opens the next
    // non-empty phase with a release
    auto complete = [&](int ph) {
        sync_release();
        int old = __hip_atomic_fetch_add(&dones[ph], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        old = __builtin_amdgcn_readfirstlane(old);
        if (old + 64 == 64 * phase_target(ph, P)) {
            // T(P-1) is the only empty phase
            const int nx = (ph + 1 == 2 * P - 1) ? ph + 2 : ph + 1;
            sync_acquire();
            sync_release();
            __hip_atomic_store(phase, nx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    auto claim = [&](int ph) -> int {
        int v = 0;
        if (lane == 0) v = atomicAdd(&claims[ph], 1);
        return __builtin_amdgcn_readfirstlane(v);
    };

    // the leaf of step t (the leader wave only), phase ph = L(t)
    auto leaf = [&](int t, int ph) {
        // tile (t,t) after the last update, into sA (column-major, pitch TP)
        if (t == 0) {
#pragma unroll
            for (int q = 0; q < 16; ++q) sA[(2 * q + lh) * TP + lr] = a_el(lr, 2 * q + lh);
        } else {
            // every load of the update in flight at once
            const float* Ug = Tt(t - 1, t);
            const float* Lg = Tt(t, t - 1);
            float* Cg = Tt(t, t);
            float v[16], a[16], cv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = gld(Ug + (int64_t)(2 * q) * ldt + offA);
#pragma unroll
            for (int q = 0; q < 16; ++q) a[q] = gld(Lg + (int64_t)(2 * q) * ldt + offA);
            if (t == 1) {
#pragma unroll
                for (int q = 0; q < 16; ++q) cv[q] = a_el(32 + lr, 32 + res_col(q, lh));
            } else {
#pragma unroll
                for (int q = 0; q < 16; ++q) cv[q] = gld(Cp(Cg, q));
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) sB[(2 * q + lh) * TP + lr] = v[q];
            const f16v_t acc = prod32([&](int k2) { return a[k2]; }, sQ(sB));
#pragma unroll
            for (int q = 0; q < 16; ++q) sA[res_col(q, lh) * TP + lr] = cv[q] - acc[q];
        }
        // LU in registers: lane r (and r + 32) holds row r.  The 31 steps are
        // unrolled, so that a step's column and the columns it sweeps (those
        // right of it) are fixed registers; the multiplier is zero for the rows
        // at or above the pivot (which then stay as they are: no branch, no
        // change of the execution mask); left of the diagonal a row then holds
        // junk, never read again, and the multipliers go to mcol (column j of
        // L, in registers).  (Rolled in blocks of four steps, for a smaller
        // code, the column read through the register index and every block's
        // columns swept from its first step on, the leaf took longer: the
        // factorisation at n = 32768 spent 21.8 against 20.8 ms in the
        // diagonal LUs.)
        // A zero or non-finite pivot spreads non-finite values into the rows
        // above the later pivots too (their multiplier zero times a
        // non-finite factor row), so the first bad pivot is recorded at its
        // own step.
        v32f x, mcol;
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            x[c] = sA[c * TP + lr];
            mcol[c] = 0.0f;
        }
        int bad = -1;
#pragma unroll
        for (int j = 0; j < 31; ++j) {
            const int lr = opaque(lane & 31);
            const float xj = x[j];
            const float pv = rl(xj, j);
            if (bad < 0 && !(pv != 0.0f && isfinite(pv))) bad = j;
            const float rp = __builtin_amdgcn_rcpf(pv);   // v_rcp_f32 (1 ulp)
            const float l = (lr > j) ? xj * rp : 0.0f;
#pragma unroll
            for (int c = j + 1; c < 32; ++c) x[c] = fmaf(-l, rl(x[c], j), x[c]);
            mcol[j] = l;
        }
        float* Cg = Tt(t, t);
        if (lh == 0) {
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                const float f = (c >= lr) ? x[c] : mcol[c];
                gst(Cg + lr + (int64_t)c * ldt, f);
                sB[c * TP + lr] = f;
            }
        }
        complete(ph);
        store_final(t, t, sB);
        // the last pivot; report the first zero / non-finite one (the
        // identity padding beyond kb has pivots 1)
        {
            const float d = rl(x[31], 31);
            if (bad < 0 && !(d != 0.0f && isfinite(d))) bad = 31;
        }
        if (bad >= 0 && 32 * t + bad < kb && lane == 0) atomicMin(info, (unsigned long long)(k + 32 * t + bad + 1));
    };

    // the inverse of the unit-lower factor of tile (t,t), as block (t&1, t&1)
    // of the column-major 64 x 64 inverse t/2 (zero above the diagonal)
    auto tile_linv = [&](int t) {
        stage_cm(sA, Tt(t, t), ldt, lr, lh);
        lds_order();
        float X[32];
        const int lro = opaque(lr);
#pragma unroll
        for (int c = 0; c < 32; ++c) X[c] = (c == lro) ? 1.0f : 0.0f;
        // by rows: X[i] = e_i - sum_{s<i} L[i][s] X[s]; row s of X is zero
        // right of s, so the sweep stops at C1 (the steps unrolled, their
        // sweeps by blocks of eight columns)
        auto linv_step = [&](int s2, auto C1) {
            constexpr int c1 = decltype(C1)::value;
            const int lr = opaque(lane & 31);
            if (lr > s2) {
                const float l = sA[s2 * TP + lr];
                // all broadcasts first (kept apart from the FMAs so that
                // the readlane results pipeline instead of alternating)
                float pv[c1];
#pragma unroll
                for (int c = 0; c < c1; ++c) pv[c] = rl(X[c], s2);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c < c1; ++c) X[c] = fmaf(-l, pv[c], X[c]);
            }
        };
#pragma unroll
        for (int s2 = 0; s2 < 31; ++s2) {
            if (s2 < 8) linv_step(s2, std::integral_constant<int, 8>());
            else if (s2 < 16) linv_step(s2, std::integral_constant<int, 16>());
            else if (s2 < 24) linv_step(s2, std::integral_constant<int, 24>());
            else linv_step(s2, std::integral_constant<int, 32>());
        }
        const int o = 32 * (t & 1);
        float* L64 = linv + (t >> 1) * 4096;
        if (lh == 0) {
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                gst(L64 + (o + lr) + 64 * (o + c), X[c]);
                if (o == 0) gst(L64 + lr + 64 * (32 + c), 0.0f);
            }
        }
    };

    // the inverse of the upper factor of tile (t,t), as block (t&1, t&1) of
    // the row-major 64 x 64 inverse t/2 (zero below the diagonal)
    auto tile_uinv = [&](int t) {
        stage_cm(sA, Tt(t, t), ldt, lr, lh);
        lds_order();
        v32f x;
        float X[32];
        const int lro = opaque(lr);
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            x[c] = sA[c * TP + lr];                 // row lr of the tile (U right of the diagonal)
            X[c] = (c == lro) ? 1.0f : 0.0f;
        }
        const float dinv = __builtin_amdgcn_rcpf(sA[lro * TP + lro]);   // 1 / U[lr][lr], as in the leaf
        // by rows, last row first: X[i] = (e_i - sum_{s>i} U[i][s] X[s]) / U[i][i];
        // row s of X is zero left of s, so the sweep starts at C0 (the steps
        // unrolled, their sweeps by blocks of eight columns)
        auto uinv_step = [&](int s2, auto C0) {
            const int lr = opaque(lane & 31);
            const float sc = (lr == s2) ? dinv : 1.0f;
#pragma unroll
            for (int c = decltype(C0)::value; c < 32; ++c) X[c] *= sc;
            const float w = x[s2];
            if (lr < s2) {
                float pv[32];
#pragma unroll
                for (int c = decltype(C0)::value; c < 32; ++c) pv[c] = rl(X[c], s2);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = decltype(C0)::value; c < 32; ++c) X[c] = fmaf(-w, pv[c], X[c]);
            }
        };
#pragma unroll
        for (int s2 = 31; s2 >= 0; --s2) {
            if (s2 >= 24) uinv_step(s2, std::integral_constant<int, 24>());
            else if (s2 >= 16) uinv_step(s2, std::integral_constant<int, 16>());
            else if (s2 >= 8) uinv_step(s2, std::integral_constant<int, 8>());
            else uinv_step(s2, std::integral_constant<int, 0>());
        }
        lds_order();
        if (lh == 0) {
#pragma unroll
            for (int c = 0; c < 32; ++c) sA[c * TP + lr] = X[c];
        }
        lds_order();
        // row-major copy, read back transposed so that the stores coalesce
        const int o = 32 * (t & 1);
        float* U64 = uinv + (t >> 1) * 4096;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = 2 * q + lh;
            gst(U64 + 64 * (o + r) + o + lr, sA[lr * TP + r]);
            if (o == 32) gst(U64 + 64 * (32 + r) + lr, 0.0f);
        }
    };

    // one task u of phase ph; it counts itself done (complete) as soon as its
    // stores to T are acknowledged
    auto task = [&](int ph, int u) {
        if (ph == NP - 2) {
            if (u < P) tile_linv(u);
            else tile_uinv(u - P);
            complete(ph);
            return;
        }
        if (ph == NP - 1) {
            if (u < P / 2) {
                // [L11 0; L21 L22]^-1 = [L11^-1 0; -L22^-1 L21 L11^-1  L22^-1]
                const int b = u;
                float* L64 = linv + b * 4096;
                const float* L21 = Tt(2 * b + 1, 2 * b);
                stage_cm(sA, L64, 64, lr, lh);
                const f16v_t y = prod32(gP(L21), sQ(sA));
#pragma unroll
                for (int q = 0; q < 16; ++q) sA[res_col(q, lh) * TP + lr] = y[q];
                const float* L22i = L64 + 32 + 64 * 32;
                const f16v_t x = prod32([=](int k2) { return gld(L22i + 128 * k2 + lr + 64 * lh); }, sQ(sA));
#pragma unroll
                for (int q = 0; q < 16; ++q) L64[(32 + lr) + 64 * res_col(q, lh)] = -x[q];
            } else {
                // [U11 U12; 0 U22]^-1 = [U11^-1  -U11^-1 U12 U22^-1; 0 U22^-1]
                const int b = u - P / 2;
                float* U64 = uinv + b * 4096;
                const float* U12 = Tt(2 * b, 2 * b + 1);
                const float* U22i = U64 + 64 * 32 + 32;
                const f16v_t z = prod32(gP(U12), [=](int k2) { return gld(U22i + 128 * k2 + 64 * lh + lr); });
#pragma unroll
                for (int q = 0; q < 16; ++q) sB[res_col(q, lh) * TP + lr] = z[q];
                stage_rm(sA, U64, 64, lr, lh);
                const f16v_t x = prod32(sP(sA), sQ(sB));
#pragma unroll
                for (int q = 0; q < 16; ++q) sA[res_col(q, lh) * TP + lr] = -x[q];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int r = 2 * q + lh;
                    U64[64 * r + 32 + lr] = sA[lr * TP + r];
                }
            }
            complete(ph);
            return;
        }
        const int t = ph / 2;
        if (ph % 2 == 0) {
            // L(t): update t-1 of trailing tile (i,j) != (t,t)
            const int w = P - t;
            const int i = t + (u + 1) % w, j = t + (u + 1) / w;
            const float* Ug = Tt(t - 1, j);
            const float* Lg = Tt(i, t - 1);
            float* Cg = Tt(i, j);
            // every global load of the task in flight at once
            float v[16], a[16], cv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = gld(Ug + (int64_t)(2 * q) * ldt + offA);
#pragma unroll
            for (int q = 0; q < 16; ++q) a[q] = gld(Lg + (int64_t)(2 * q) * ldt + offA);
            if (t == 1) {
#pragma unroll
                for (int q = 0; q < 16; ++q) cv[q] = a_el(32 * i + lr, 32 * j + res_col(q, lh));
            } else {
#pragma unroll
                for (int q = 0; q < 16; ++q) cv[q] = gld(Cp(Cg, q));
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) sA[(2 * q + lh) * TP + lr] = v[q];
            const f16v_t acc = prod32([&](int k2) { return a[k2]; }, sQ(sA));
#pragma unroll
            for (int q = 0; q < 16; ++q) gst(Cp(Cg, q), cv[q] - acc[q]);
            complete(ph);
            return;
        }
        // T(t), by substitution against the factored tile (t,t), staged in
        // sA with pitch SP so that four consecutive factor entries are one
        // 16-byte LDS read (the same address in every lane: a broadcast)
        const int w = P - 1 - t;
        const float* Fg = Tt(t, t);
        const int lo = lr, ho = lh;
        float b[32];
        if (u < w) {
            // tile (i,t) <- tile (i,t) U_tt^-1: X U = B row by row, lane r
            // holding row r; U is staged row-major (sA[s*SP + c] = U[s][c])
            float* Xg = Tt(t + 1 + u, t);
            float f[16];
            if (t == 0) {
#pragma unroll
                for (int c = 0; c < 32; ++c) b[c] = a_el(32 * (1 + u) + lo, c);
            } else {
#pragma unroll
                for (int c = 0; c < 32; ++c) b[c] = gld(Xg + lo + (int64_t)c * ldt);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) f[q] = gld(Fg + lo + (int64_t)(2 * q + ho) * ldt);
#pragma unroll
            for (int q = 0; q < 16; ++q) sA[lo * SP + 2 * q + ho] = f[q];
            lds_order();
#pragma unroll
            for (int s2 = 0; s2 < 32; ++s2) {
                float urow[32];
#pragma unroll
                for (int m = s2 / 4; m < 8; ++m) {
                    const float4 v = *reinterpret_cast<const float4*>(sA + s2 * SP + 4 * m);
                    urow[4 * m] = v.x;
                    urow[4 * m + 1] = v.y;
                    urow[4 * m + 2] = v.z;
                    urow[4 * m + 3] = v.w;
                }
                b[s2] *= __builtin_amdgcn_rcpf(urow[s2]);
#pragma unroll
                for (int c = s2 + 1; c < 32; ++c) b[c] = fmaf(-b[s2], urow[c], b[c]);
                // the step completes here: one factor row live at a time
                pin(b[s2]);
#pragma unroll
                for (int c = s2 + 1; c < 32; ++c) pin(b[c]);
            }
            lds_order();
            if (ho == 0) {
#pragma unroll
                for (int c = 0; c < 32; ++c) sB[c * TP + lo] = b[c];
            }
            lds_order();
#pragma unroll
            for (int q = 0; q < 16; ++q) gst(Xg + lo + (int64_t)(2 * q + ho) * ldt, sB[(2 * q + ho) * TP + lo]);
            complete(ph);
            store_final(t + 1 + u, t, sB);
        } else {
            // tile (t,j) <- L_tt^-1 tile (t,j): L Y = B column by column, lane
            // r holding column r; the unit-lower L is staged column-major
            // (sA[q*SP + s] = L[s][q])
            const int j = t + 1 + (u - w);
            float* Yg = Tt(t, j);
            float f[16];
            if (t == 0) {
#pragma unroll
                for (int q = 0; q < 16; ++q) sB[(2 * q + ho) * TP + lo] = a_el(lo, 32 * j + 2 * q + ho);
            } else {
                stage_cm(sB, Yg, ldt, lo, ho);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) f[q] = gld(Fg + lo + (int64_t)(2 * q + ho) * ldt);
#pragma unroll
            for (int q = 0; q < 16; ++q) sA[(2 * q + ho) * SP + lo] = f[q];
            lds_order();
#pragma unroll
            for (int s2 = 0; s2 < 32; ++s2) b[s2] = sB[lo * TP + s2];
#pragma unroll
            for (int q = 0; q < 31; ++q) {
                float lcol[32];
#pragma unroll
                for (int m = (q + 1) / 4; m < 8; ++m) {
                    const float4 v = *reinterpret_cast<const float4*>(sA + q * SP + 4 * m);
                    lcol[4 * m] = v.x;
                    lcol[4 * m + 1] = v.y;
                    lcol[4 * m + 2] = v.z;
                    lcol[4 * m + 3] = v.w;
                }
#pragma unroll
                for (int s2 = q + 1; s2 < 32; ++s2) b[s2] = fmaf(-lcol[s2], b[q], b[s2]);
#pragma unroll
                for (int s2 = q + 1; s2 < 32; ++s2) pin(b[s2]);
            }
            lds_order();
            if (ho == 0) {
#pragma unroll
                for (int s2 = 0; s2 < 32; ++s2) sB[lo * TP + s2] = b[s2];
            }
            lds_order();
#pragma unroll
            for (int q = 0; q < 16; ++q) gst(Yg + lo + (int64_t)(2 * q + ho) * ldt, sB[(2 * q + ho) * TP + lo]);
            complete(ph);
            store_final(t, j, sB);
        }
    };

    // every wave: from the open phase on, take part in each phase in turn
    int ph = ild(phase);
    for (; ph < NP; ++ph) {
        if (phase_target(ph, P) == 0) continue;
        if (!wait_phase(ph)) return;
        if (leader && is_lphase(ph, P)) {
            refresh();
            leaf(ph / 2, ph);
        }
        const int nclaim = phase_claims(ph, P);
        for (;;) {
            const int u = claim(ph);
            if (u >= nclaim) break;
            refresh();
            task(ph, u);   // counts itself done
        }
    }
}

size_t diag_lu_smem() { return (size_t)(2 * DW) * TILE_F * sizeof(float); }
size_t diag_sync_words() { return 1 + 2 * NPMAX; }

// most work-groups cooperating on one diagonal block
#ifndef MXP_DIAG_WGS
#define MXP_DIAG_WGS 24
#endif

template <int ST>
static hipError_t diag_lu_typed(const DiagCall* calls, int count, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_diag_lu<ST>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)diag_lu_smem());
    if (attr) return attr;
    DiagGroup grp;
    int wmax = 1;
    for (int i = 0; i < count; ++i) {
        const DiagCall& c = calls[i];
        DiagOne& g = grp.g[i];
        g.A = c.A; g.lda = c.lda; g.k = c.k; g.kb = c.kb; g.kbp = c.kbp; g.ldt = c.ldt;
        g.T = c.T; g.Trm = c.Trm; g.linv = c.linv; g.uinv = c.uinv; g.sync = c.sync; g.info = c.info;
        // helpers scale with the work: two work-groups per tile column, at
        // most 24 (a 512 block: one leader work-group and 23 helpers; its
        // early update phases have up to 224 tile tasks).  Measured at
        // n = 32768: 16 / 24 / 32 work-groups 45.1 / 44.8 / 45.1 ms for the
        // factorisation; with the unrolled leaf 421.9 / 421.7 / 418.3
        // TFLOP/s for the solve (mean of two, one box)
        const int P = c.kbp / 32;
        g.wgs = P < 1 ? 1 : (2 * P > MXP_DIAG_WGS ? MXP_DIAG_WGS : 2 * P);
        wmax = g.wgs > wmax ? g.wgs : wmax;
    }
    grp.count = count;
    k_diag_lu<ST><<<dim3(wmax, count), DT, diag_lu_smem(), s>>>(grp);
    return hipGetLastError();
}

hipError_t diag_lu_group(int store, const DiagCall* calls, int count, hipStream_t s) {
    if (count < 1 || count > GEMM_GROUP_MAX) return hipErrorInvalidValue;
    for (int i = 0; i < count; ++i) {
        const DiagCall& c = calls[i];
        if (c.kb < 1 || c.kbp % 64 || c.kbp > c.ldt || c.kb > c.kbp || c.kbp > 1024) return hipErrorInvalidValue;
    }
    switch (store) {
    case F32: return diag_lu_typed<F32>(calls, count, s);
    case F16: return diag_lu_typed<F16>(calls, count, s);
    case BF16: return diag_lu_typed<BF16>(calls, count, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t diag_lu(int store, void* A, int64_t lda, int64_t k, int kb, int kbp, float* T, float* Trm, int ldt,
                   float* linv, float* uinv, int* sync, unsigned long long* info, hipStream_t s) {
    DiagCall c{A, lda, k, kb, kbp, ldt, T, Trm, linv, uinv, sync, info};
    return diag_lu_group(store, &c, 1, s);
}

}  // namespace mxp
