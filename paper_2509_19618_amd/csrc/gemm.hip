// gemm.hip -- the Schur-complement update of the blocked LU on the matrix
// cores (paper: "Algorithmic Framework", Figure 1: A22 <- A22 - A21 A11^-1 A12
// with 16-bit (here also 8-bit) inputs and 32-bit accumulation).
//
//   C (M x N, storage format, column-major, ldc)
//     <- C - diag(inv_sa) (Aq Bq^T) diag(inv_sb)
//   Aq: M x K operand (K-major rows), Bq: N x K operand (K-major rows),
//   inv_sa / inv_sb: one power-of-two factor per 32 rows / 32 columns.
//
// The accumulators start at zero and hold sum Aq Bq^T in FP32; the result
// C - acc * (inv_sa inv_sb) is rounded once to the storage format.
//
// An update may have a second K segment: the operands of the next block step
// with factors of their own (the updates of two consecutive steps merged,
// which halves the C traffic per flop).  At the segment boundary each 32 x 32
// accumulator block is multiplied by (inv_sa inv_sb) / (inv_sa2 inv_sb2), a
// power of two (exact), the second segment accumulates onto it, and the
// result is C - acc * (inv_sa2 inv_sb2), rounded once.
//
// Work-groups are dispatched round-robin over the 8 XCDs; the tile order
// gives every XCD a contiguous range of tiles, walked in groups of 8 tile
// rows so that the operand panels in flight on an XCD fit its L2.
#include "common.hpp"
#include "kernels.hpp"

namespace mxp {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i2v __attribute__((ext_vector_type(2)));

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
        // operand formats 0/0 = fp8 e4m3 for both; E8M0 block scales of 1.0
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x, y, c, 0, 0, 0, 0x7f7f7f7f, 0, 0x7f7f7f7f);
    }
};
template <> struct Mfma<F32> {
    static constexpr int KB = 8;   // 2 floats
    static MXP_DEV f16v run(const char* a, const char* b, f16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(*(const float*)a, *(const float*)b, c, 0, 0, 0);
    }
};

// four consecutive storage elements of one column <-> four floats
template <int ST> struct Quad;
template <> struct Quad<F32> {
    static MXP_DEV void load(const float* p, float v[4]) {
        i4v x = *(const i4v*)p;
        for (int q = 0; q < 4; ++q) v[q] = __int_as_float(x[q]);
    }
    static MXP_DEV void store(float* p, const float v[4]) {
        i4v x = {__float_as_int(v[0]), __float_as_int(v[1]), __float_as_int(v[2]), __float_as_int(v[3])};
        *(i4v*)p = x;
    }
};
template <> struct Quad<F16> {
    static MXP_DEV void load(const half_t* p, float v[4]) {
        i2v x = *(const i2v*)p;
        const half_t* h = (const half_t*)&x;
        for (int q = 0; q < 4; ++q) v[q] = (float)h[q];
    }
    static MXP_DEV void store(half_t* p, const float v[4]) {
        half_t h[4];
        for (int q = 0; q < 4; ++q) h[q] = (half_t)v[q];
        *(i2v*)p = *(const i2v*)h;
    }
};
template <> struct Quad<BF16> {
    static MXP_DEV void load(const bf16_t* p, float v[4]) {
        i2v x = *(const i2v*)p;
        const bf16_t* h = (const bf16_t*)&x;
        for (int q = 0; q < 4; ++q) v[q] = bf16_bits_to_f32(h[q]);
    }
    static MXP_DEV void store(bf16_t* p, const float v[4]) {
        bf16_t h[4];
        for (int q = 0; q < 4; ++q) h[q] = f32_to_bf16_bits(v[q]);
        *(i2v*)p = *(const i2v*)h;
    }
};

// Work-group tile TMv x TN (TMv = 256 or 128, TN = 128), 4 waves in a 2 x 2
// grid, each wave (TMv/2) x 64 (blocks of 32 x 32, accumulators in AGPRs).
// With TMv = 256 two work-groups share a CU (at most 256 registers per wave,
// 72 KB of LDS each), so that one work-group's epilogue overlaps the other's
// MFMA loop; TMv = 128 gives twice as many tiles for small trailing matrices.
constexpr int TN = 128;
constexpr int GBK = 64;            // K bytes per stage
#ifndef MXP_NBUF
#define MXP_NBUF 3
#endif
constexpr int NBUF = MXP_NBUF;     // stages in LDS: two copies in flight while one is read
constexpr int GCH = GBK / 16;      // 16-byte chunks per operand row
constexpr int SB = TN * GBK;       // bytes of one B stage
constexpr int GGROUP = 8;          // tile rows per group in the tile order
#ifndef MXP_GGROUP2
#define MXP_GGROUP2 4
#endif
constexpr int GGROUP2 = MXP_GGROUP2;   // the same for two-segment updates (twice the operand bytes per tile row)

// Direct global->LDS copy of 16 bytes per lane: lane L lands at l + 16 L
// (l is wave-uniform).  gfx950 global_load_lds_dwordx4.
MXP_DEV void dma16(const char* g, char* l) {
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)g,
                                     (void __attribute__((address_space(3)))*)l, 16, 0, 0);
}
// s_waitcnt vmcnt(N) (expcnt / lgkmcnt not waited); N < 64
template <int N> MXP_DEV void wait_vm() {
    static_assert(N < 64, "vmcnt has six bits");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | (0x7 << 4) | (0xF << 8) | ((N >> 4) << 14));
}
// wait_vm<y NIS + (c ? NC : 0)> for a wave-uniform y <= Y
template <int NIS, int NC, int Y> MXP_DEV void wait_case(int y, bool c) {
    if constexpr (Y >= 0) {
        if (y == Y) {
            if (c) wait_vm<Y * NIS + NC>();
            else wait_vm<Y * NIS>();
            return;
        }
        wait_case<NIS, NC, Y - 1>(y, c);
    }
}


// c - a d with d a power of two (a d exact): one rounding to FP32; the
// rounding to the storage format stays a separate step in every epilogue
// (the compiler would otherwise fuse some of them into one FP16 rounding,
// and the two epilogues would differ in the last bit)
MXP_DEV float sub_scaled(float c, float a, float d) {
    float v = __builtin_fmaf(-a, d, c);
    asm volatile("" : "+v"(v));
    return v;
}

// The 16-byte chunks of an operand row (64 bytes) are XOR-swizzled by a key
// of the row, so that the 16-byte fragment reads of consecutive rows (one
// row per lane) spread over the LDS banks.  A row spans 16 of the 64 banks
// (4 bytes each), so rows r, r+4, r+8, r+12 fall on the same banks; the key
// (row / 4) mod 4 gives them four different chunk positions.  Measured with
// SQ_LDS_BANK_CONFLICT on the MI355X: 21x fewer conflict cycles than the key
// row mod 4, and 5 % more update throughput.
MXP_DEV int swz_key(int row) { return (row >> 2) & (GCH - 1); }
// byte offset of (row, byte b) in an operand stage
MXP_DEV int swz(int row, int b) { return row * GBK + ((((b >> 4) ^ swz_key(row)) << 4) | (b & 15)); }

template <int OP> struct Frag;
template <> struct Frag<F16> {
    typedef h8v T;
    static MXP_DEV T ld(const char* s, int row, int b) { return *(const h8v*)(s + swz(row, b)); }
    static MXP_DEV f16v mma(T a, T b, f16v c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};
template <> struct Frag<BF16> {
    typedef b8v T;
    static MXP_DEV T ld(const char* s, int row, int b) { return *(const b8v*)(s + swz(row, b)); }
    static MXP_DEV f16v mma(T a, T b, f16v c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};
template <> struct Frag<F32> {
    typedef float T;
    static MXP_DEV T ld(const char* s, int row, int b) { return *(const float*)(s + swz(row, b)); }
    static MXP_DEV f16v mma(T a, T b, f16v c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
};
template <> struct Frag<F8> {
    typedef i8v T;
    static MXP_DEV T ld(const char* s, int row, int b) {
        i4v a0 = *(const i4v*)(s + swz(row, b)), a1 = *(const i4v*)(s + swz(row, b + 16));
        i8v x = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
        return x;
    }
    // operand formats 0/0 = fp8 e4m3 for both; E8M0 block scales of 1.0
    static MXP_DEV f16v mma(T a, T b, f16v c) {
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0x7f7f7f7f, 0, 0x7f7f7f7f);
    }
};

// One launch serves a group of independent updates (one per request of the
// solve server, or a single one): the tiles of the group's updates are
// numbered one after another and every work-group finds its update by its
// tile number.  Passed by value (kernel arguments).
struct GemmOne {
    void* C;
    int64_t ldc, M, N;
    const char* Aq;
    const char* Bq;
    const float* inv_sa;
    const float* inv_sb;
    const char* Aq2;                 // second segment (K2 > 0)
    const char* Bq2;
    const float* inv_sa2;
    const float* inv_sb2;
    int K, K2, tiles_m, tiles_n, tile_end, vec_ok;
};
struct GemmGroup {
    GemmOne g[GEMM_DESC_MAX];
    int count, per_xcd;
};

// Operands: K-major rows, copied GBK bytes of K per stage straight into
// XOR-swizzled LDS buffers (no staging registers), NBUF stages deep; each
// k-step reads its fragments from LDS (the other work-group on the SIMD
// covers their latency).  Epilogue, full tiles with 16-bit C: the freed LDS
// holds the C tile (read and written with coalesced 16-byte accesses, TMv*2
// bytes per column), updated in place in the MFMA layout; the first half of
// the tile is loaded into registers at the first stage, so that its HBM
// reads overlap the MFMA loop (the whole tile would not fit beside the
// accumulators), the second half in the epilogue.  Other tiles update C
// directly with guarded accesses.
template <int OP, int ST, int TMv>
__global__ __launch_bounds__(256, 2) void k_gemm_update(const GemmGroup grp) {
    typedef typename Store<ST>::T CT;
    typedef typename Frag<OP>::T FT;
    constexpr int SA = TMv * GBK;          // bytes of one A stage
    constexpr int WR = TMv / 2;            // rows of a wave's tile
    constexpr int NA = TMv / 64;           // 32-row blocks of a wave's tile
    constexpr int KB = Mfma<OP>::KB;
    constexpr int NKS = GBK / KB;          // k-steps per stage
    constexpr int RPI = 64 / GCH;          // operand rows per 1 KB copy instruction
    constexpr int NIA = TMv / RPI / 4, NIB = TN / RPI / 4;   // copy instructions per wave and stage
    constexpr int NIS = NIA + NIB;
    constexpr int CP = TMv * (int)sizeof(CT) + 16;  // LDS pitch of a C column in the epilogue
    extern __shared__ __attribute__((aligned(16))) char lds[];
    char* sA = lds;
    char* sB = lds + NBUF * SA;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    // work-group j of XCD x (x = blockIdx % 8) takes tile x*per_xcd + j of its XCD's contiguous range
    const int xcd = (int)(blockIdx.x % 8);
    const int glin = xcd * grp.per_xcd + (int)(blockIdx.x / 8);
    const int total = grp.g[grp.count - 1].tile_end;
    if (glin >= min((xcd + 1) * grp.per_xcd, total)) return;
    int d = 0;
    while (glin >= grp.g[d].tile_end) ++d;
    const GemmOne& G = grp.g[d];
    CT* C = (CT*)G.C;
    const int64_t ldc = G.ldc, M = G.M, N = G.N;
    const int tiles_m = G.tiles_m, tiles_n = G.tiles_n, vec_ok = G.vec_ok;
    // the epilogue's factors: those of the last segment
    const float* __restrict__ inv_sa = G.K2 ? G.inv_sa2 : G.inv_sa;
    const float* __restrict__ inv_sb = G.K2 ? G.inv_sb2 : G.inv_sb;
    const int lin = glin - (d > 0 ? grp.g[d - 1].tile_end : 0);
    const int gg = G.K2 ? GGROUP2 : GGROUP;
    const int group_size = gg * tiles_n;
    const int first_m = (lin / group_size) * gg;
    const int gm = (tiles_m - first_m) < gg ? (tiles_m - first_m) : gg;
    const int tm = first_m + (lin % group_size) % gm;
    const int tn = (lin % group_size) / gm;
    const int64_t row0 = (int64_t)tm * TMv, col0 = (int64_t)tn * TN;
    constexpr int eb = sizeof(typename Operand<OP>::T);
    const int64_t Kb1 = (int64_t)G.K * eb, Kb2 = (int64_t)G.K2 * eb;
    const char* gA1 = G.Aq + row0 * Kb1;
    const char* gB1 = G.Bq + col0 * Kb1;
    const char* gA2 = G.K2 ? G.Aq2 + row0 * Kb2 : gA1;
    const char* gB2 = G.K2 ? G.Bq2 + col0 * Kb2 : gB1;
    const int nst1 = (int)(Kb1 / GBK);
    const int nst = nst1 + (int)(Kb2 / GBK);
    const int lr = lane & 31, lh = lane >> 5;
    const int l_row = lane / GCH, l_pch = lane % GCH;
    auto issue = [&](int st) {
        const int buf = st % NBUF;
        const bool s2 = st >= nst1;                           // wave-uniform
        const char* gA = s2 ? gA2 : gA1;
        const char* gB = s2 ? gB2 : gB1;
        const int64_t Kbytes = s2 ? Kb2 : Kb1;
        const int64_t ko = (int64_t)(s2 ? st - nst1 : st) * GBK;
#pragma unroll
        for (int i = 0; i < NIA; ++i) {
            const int j = wave * NIA + i;                     // 1 KB slice of the stage
            const int row = j * RPI + l_row;
            const int lch = l_pch ^ swz_key(row);            // logical chunk stored at this lane's slot
            dma16(gA + (int64_t)row * Kbytes + ko + lch * 16, sA + buf * SA + j * 1024);
        }
#pragma unroll
        for (int i = 0; i < NIB; ++i) {
            const int j = wave * NIB + i;
            const int row = j * RPI + l_row;
            const int lch = l_pch ^ swz_key(row);
            dma16(gB + (int64_t)row * Kbytes + ko + lch * 16, sB + buf * SB + j * 1024);
        }
    };
    f16v acc[NA][2];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    const bool full = vec_ok && (row0 + TMv <= M) && (col0 + TN <= N);
    constexpr bool c16 = sizeof(CT) == 2;
    const bool cpre = c16 && full;
    constexpr int COLB = TMv * 2;          // bytes of a tile column
    constexpr int LPC = COLB / 16;         // lanes per column
    constexpr int CPI = 64 / LPC;          // columns per wave instruction
    constexpr int NIT = TN / 4 / CPI;      // instructions per wave
    const int lc = lane / LPC, lo = (lane % LPC) * 16;
    i4v xv[NIT];                           // the C tile, 16 bytes per register quad
#pragma unroll
    for (int st = 0; st < NBUF - 1; ++st)
        if (st < nst) issue(st);
    for (int st = 0; st < nst; ++st) {
        // stage st has landed when at most the younger stages' copies are
        // outstanding, and the C loads while they are younger than stage st
        // (issued at stage 0, after the copies of stages up to NBUF - 1)
        const int younger = (NBUF - 2) < (nst - 1 - st) ? (NBUF - 2) : (nst - 1 - st);
        const bool cy = cpre && st > 0 && st <= NBUF - 1;
        wait_case<NIS, NIT / 2, NBUF - 2>(younger, cy);
        __syncthreads();                  // stage st visible to all; stage st-1's buffer free
        if (st + NBUF - 1 < nst) issue(st + NBUF - 1);
        if (cpre && st == 0) {
#pragma unroll
            for (int it = 0; it < NIT / 2; ++it) {
                const int c = (wave * NIT + it) * CPI + lc;
                xv[it] = __builtin_nontemporal_load((const i4v*)((const char*)(C + row0 + (col0 + c) * ldc) + lo));
            }
        }
        if (st == nst1 && st > 0) {
            // first stage of the second segment: the first segment's sums to its scale
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int64_t ra = (row0 + wm * WR + a * 32) / 32;
                const float fa = G.inv_sa[ra] / G.inv_sa2[ra];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int64_t cb = (col0 + wn * 64 + b * 32) / 32;
                    const float f = fa * (G.inv_sb[cb] / G.inv_sb2[cb]);
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[a][b][r] *= f;
                }
            }
        }
        const char* A0 = sA + (st % NBUF) * SA;
        const char* B0 = sB + (st % NBUF) * SB;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            FT ac[NA], bc[2];
            const int boff = ks * KB + lh * (KB / 2);
#pragma unroll
            for (int a = 0; a < NA; ++a) ac[a] = Frag<OP>::ld(A0, wm * WR + a * 32 + lr, boff);
#pragma unroll
            for (int b = 0; b < 2; ++b) bc[b] = Frag<OP>::ld(B0, wn * 64 + b * 32 + lr, boff);
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = Frag<OP>::mma(ac[a], bc[b], acc[a][b]);
        }
    }
    if constexpr (sizeof(CT) == 2) {
        if (full) {
            __syncthreads();                       // operand buffers no longer read
#pragma unroll
            for (int it = NIT / 2; it < NIT; ++it) {
                const int c = (wave * NIT + it) * CPI + lc;
                xv[it] = __builtin_nontemporal_load((const i4v*)((const char*)(C + row0 + (col0 + c) * ldc) + lo));
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int c = (wave * NIT + it) * CPI + lc;
                *(i4v*)(lds + c * CP + lo) = xv[it];
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const float ia = inv_sa[(row0 + wm * WR + a * 32) / 32];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const float dd = ia * inv_sb[(col0 + wn * 64 + b * 32) / 32];
                    const int c = wn * 64 + b * 32 + lr;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        CT* p = (CT*)(lds + c * CP) + wm * WR + a * 32 + 8 * g + 4 * lh;
                        float cv[4], v[4];
                        Quad<ST>::load(p, cv);
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[q] = sub_scaled(cv[q], acc[a][b][g * 4 + q], dd);
                        Quad<ST>::store(p, v);
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int c = (wave * NIT + it) * CPI + lc;
                i4v x = *(const i4v*)(lds + c * CP + lo);
                __builtin_nontemporal_store(x, (i4v*)((char*)(C + row0 + (col0 + c) * ldc) + lo));
            }
            return;
        }
    }
    // direct epilogue (FP32 storage, edge tiles): C - acc * d, quads of 4 rows
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        const int64_t rb = row0 + wm * WR + a * 32;
        const float ia = inv_sa[rb / 32];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t cb = col0 + wn * 64 + b * 32;
            const float dd = ia * inv_sb[cb / 32];
            const int64_t col = cb + lr;
            if (col >= N) continue;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t r = rb + 8 * g + 4 * lh;
                CT* p = C + r + col * ldc;
                float c[4], v[4];
                const bool quad = vec_ok && r + 3 < M;
                if (quad) Quad<ST>::load(p, c);
                else
                    for (int q = 0; q < 4; ++q) c[q] = (r + q < M) ? Store<ST>::load(p, q) : 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = sub_scaled(c[q], acc[a][b][g * 4 + q], dd);
                if (quad) Quad<ST>::store(p, v);
                else
                    for (int q = 0; q < 4; ++q)
                        if (r + q < M) p[q] = Store<ST>::from_f32(v[q]);
            }
        }
    }
}

template <int TMv>
static constexpr int gemm_lds_bytes() {
    return NBUF * (TMv * GBK + SB) > TN * (TMv * 2 + 16) ? NBUF * (TMv * GBK + SB) : TN * (TMv * 2 + 16);
}

int gemm_tile_rows(int tile) { return tile == GEMM_TILE_128 ? 128 : 256; }

template <int OP, int ST, int TMv>
static hipError_t gemm_typed(const GemmCall* calls, int count, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_gemm_update<OP, ST, TMv>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       gemm_lds_bytes<TMv>());
    if (attr) return attr;
    GemmGroup grp;
    int total = 0, used = 0;
    for (int i = 0; i < count; ++i) {
        const GemmCall& c = calls[i];
        if (c.M <= 0 || c.N <= 0) continue;
        GemmOne& g = grp.g[used++];
        g.C = c.C; g.ldc = c.ldc; g.M = c.M; g.N = c.N;
        g.Aq = (const char*)c.Aq; g.Bq = (const char*)c.Bq; g.inv_sa = c.inv_sa; g.inv_sb = c.inv_sb;
        g.K = c.K;
        g.K2 = c.K2;
        g.Aq2 = (const char*)c.Aq2; g.Bq2 = (const char*)c.Bq2; g.inv_sa2 = c.inv_sa2; g.inv_sb2 = c.inv_sb2;
        g.tiles_m = (int)((c.M + TMv - 1) / TMv);
        g.tiles_n = (int)((c.N + TN - 1) / TN);
        total += g.tiles_m * g.tiles_n;
        g.tile_end = total;
        // vectorised C access needs 16-byte aligned columns
        g.vec_ok = ((c.ldc * (int64_t)sizeof(typename Store<ST>::T)) % 16 == 0 && (((uintptr_t)c.C) % 16) == 0) ? 1
                                                                                                               : 0;
    }
    if (!used) return hipSuccess;
    grp.count = used;
    grp.per_xcd = (total + 7) / 8;
    k_gemm_update<OP, ST, TMv><<<8 * grp.per_xcd, 256, gemm_lds_bytes<TMv>(), s>>>(grp);
    return hipGetLastError();
}

hipError_t gemm_group(int update, int store, int tile, const GemmCall* calls, int count, hipStream_t s) {
    if (count < 1 || count > GEMM_DESC_MAX) return hipErrorInvalidValue;
    for (int i = 0; i < count; ++i) {
        const GemmCall& c = calls[i];
        if (c.K < 1 || (c.K * dtype_bytes(update)) % GBK || c.K2 < 0 || (c.K2 * dtype_bytes(update)) % GBK ||
            (c.K2 && (!c.Aq2 || !c.Bq2 || !c.inv_sa2 || !c.inv_sb2)))
            return hipErrorInvalidValue;
    }
#define GCASE(U, S)                                                                                      \
    if (update == U && store == S)                                                                       \
        return tile == GEMM_TILE_128 ? gemm_typed<U, S, 128>(calls, count, s) : gemm_typed<U, S, 256>(calls, count, s)
    GCASE(F32, F32);
    GCASE(F16, F16);
    GCASE(BF16, BF16);
    GCASE(F8, F16);
    GCASE(F8, BF16);
    GCASE(F16, F32);
    GCASE(BF16, F32);
#undef GCASE
    return hipErrorInvalidValue;
}

hipError_t gemm_update(int update, int store, void* C, int64_t ldc, int64_t M, int64_t N, int K, const void* Aq,
                       const void* Bq, const float* inv_sa, const float* inv_sb, hipStream_t s, int tile) {
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmCall c{C, ldc, M, N, K, Aq, Bq, inv_sa, inv_sb};
    return gemm_group(update, store, tile, &c, 1, s);
}

}  // namespace mxp
