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

// Work-group tile TM x TN = 256 x 128, 4 waves in a 2 x 2 grid, each wave
// 128 x 64 (8 blocks of 32 x 32, accumulators in AGPRs).  Two work-groups
// share a CU (at most 256 registers per wave, 72 KB of LDS each), so that
// one work-group's epilogue overlaps the other's MFMA loop.
constexpr int TM = 256, TN = 128;
constexpr int GBK = 64;            // K bytes per stage
constexpr int NBUF = 3;            // stages in LDS: two copies in flight while one is read
constexpr int GCH = GBK / 16;      // 16-byte chunks per operand row
constexpr int SA = TM * GBK, SB = TN * GBK;   // bytes of one A / B stage
constexpr int GGROUP = 8;          // tile rows per group in the tile order

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


// byte offset of (row, byte b) in an operand stage: 16-byte chunks XOR-swizzled by row
MXP_DEV int swz(int row, int b) { return row * GBK + ((((b >> 4) ^ (row & (GCH - 1))) << 4) | (b & 15)); }

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

// Operands: K-major rows, copied GBK bytes of K per stage straight into
// XOR-swizzled LDS buffers (no staging registers), NBUF stages deep; each
// k-step reads its fragments from LDS (the other work-group on the SIMD
// covers their latency).  Epilogue, full tiles with 16-bit C: the freed LDS
// holds the C tile (read and written with coalesced 16-byte accesses, 512
// bytes per column), updated in place in the MFMA layout; the first half of
// the tile is loaded into registers at the first stage, so that its HBM
// reads overlap the MFMA loop (the whole tile would not fit beside the
// accumulators), the second half in the epilogue.  Other tiles update C
// directly with guarded accesses.
template <int OP, int ST>
__global__ __launch_bounds__(256, 2) void k_gemm_update(typename Store<ST>::T* C, int64_t ldc, int64_t M, int64_t N,
                                                        int K, const char* __restrict__ Aq,
                                                        const char* __restrict__ Bq,
                                                        const float* __restrict__ inv_sa,
                                                        const float* __restrict__ inv_sb, int tiles_m, int tiles_n,
                                                        int per_xcd, int vec_ok) {
    typedef typename Store<ST>::T CT;
    typedef typename Frag<OP>::T FT;
    constexpr int KB = Mfma<OP>::KB;
    constexpr int NKS = GBK / KB;          // k-steps per stage
    constexpr int RPI = 64 / GCH;          // operand rows per 1 KB copy instruction
    constexpr int NIA = TM / RPI / 4, NIB = TN / RPI / 4;   // copy instructions per wave and stage
    constexpr int NIS = NIA + NIB;
    constexpr int CP = TM * (int)sizeof(CT) + 16;  // LDS pitch of a C column in the epilogue
    extern __shared__ __attribute__((aligned(16))) char lds[];
    char* sA = lds;
    char* sB = lds + NBUF * SA;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    // work-group j of XCD x (x = blockIdx % 8) takes tile x*per_xcd + j of its XCD's contiguous range
    const int xcd = (int)(blockIdx.x % 8);
    const int lin = xcd * per_xcd + (int)(blockIdx.x / 8);
    if (lin >= min((xcd + 1) * per_xcd, tiles_m * tiles_n)) return;
    const int group_size = GGROUP * tiles_n;
    const int first_m = (lin / group_size) * GGROUP;
    const int gm = (tiles_m - first_m) < GGROUP ? (tiles_m - first_m) : GGROUP;
    const int tm = first_m + (lin % group_size) % gm;
    const int tn = (lin % group_size) / gm;
    const int64_t row0 = (int64_t)tm * TM, col0 = (int64_t)tn * TN;
    constexpr int eb = sizeof(typename Operand<OP>::T);
    const int64_t Kbytes = (int64_t)K * eb;
    const char* gA = Aq + row0 * Kbytes;
    const char* gB = Bq + col0 * Kbytes;
    const int nst = (int)(Kbytes / GBK);
    const int lr = lane & 31, lh = lane >> 5;
    const int l_row = lane / GCH, l_pch = lane % GCH;
    auto issue = [&](int st) {
        const int buf = st % NBUF;
#pragma unroll
        for (int i = 0; i < NIA; ++i) {
            const int j = wave * NIA + i;                     // 1 KB slice of the stage
            const int row = j * RPI + l_row;
            const int lch = l_pch ^ (row & (GCH - 1));        // logical chunk stored at this lane's slot
            dma16(gA + (int64_t)row * Kbytes + (int64_t)st * GBK + lch * 16, sA + buf * SA + j * 1024);
        }
#pragma unroll
        for (int i = 0; i < NIB; ++i) {
            const int j = wave * NIB + i;
            const int row = j * RPI + l_row;
            const int lch = l_pch ^ (row & (GCH - 1));
            dma16(gB + (int64_t)row * Kbytes + (int64_t)st * GBK + lch * 16, sB + buf * SB + j * 1024);
        }
    };
    f16v acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    const bool full = vec_ok && (row0 + TM <= M) && (col0 + TN <= N);
    constexpr bool c16 = sizeof(CT) == 2;
    const bool cpre = c16 && full;
    constexpr int COLB = TM * 2;           // bytes of a tile column
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
        const char* A0 = sA + (st % NBUF) * SA;
        const char* B0 = sB + (st % NBUF) * SB;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            FT ac[4], bc[2];
            const int boff = ks * KB + lh * (KB / 2);
#pragma unroll
            for (int a = 0; a < 4; ++a) ac[a] = Frag<OP>::ld(A0, wm * 128 + a * 32 + lr, boff);
#pragma unroll
            for (int b = 0; b < 2; ++b) bc[b] = Frag<OP>::ld(B0, wn * 64 + b * 32 + lr, boff);
#pragma unroll
            for (int a = 0; a < 4; ++a)
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
            for (int a = 0; a < 4; ++a) {
                const float ia = inv_sa[(row0 + wm * 128 + a * 32) / 32];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const float d = ia * inv_sb[(col0 + wn * 64 + b * 32) / 32];
                    const int c = wn * 64 + b * 32 + lr;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        CT* p = (CT*)(lds + c * CP) + wm * 128 + a * 32 + 8 * g + 4 * lh;
                        float cv[4], v[4];
                        Quad<ST>::load(p, cv);
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[q] = cv[q] - acc[a][b][g * 4 + q] * d;
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
    for (int a = 0; a < 4; ++a) {
        const int64_t rb = row0 + wm * 128 + a * 32;
        const float ia = inv_sa[rb / 32];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t cb = col0 + wn * 64 + b * 32;
            const float d = ia * inv_sb[cb / 32];
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
                for (int q = 0; q < 4; ++q) v[q] = c[q] - acc[a][b][g * 4 + q] * d;
                if (quad) Quad<ST>::store(p, v);
                else
                    for (int q = 0; q < 4; ++q)
                        if (r + q < M) p[q] = Store<ST>::from_f32(v[q]);
            }
        }
    }
}

static constexpr int gemm_lds_bytes() {
    return NBUF * (SA + SB) > TN * (TM * 2 + 16) ? NBUF * (SA + SB) : TN * (TM * 2 + 16);
}

template <int OP, int ST>
static hipError_t gemm_typed(void* C, int64_t ldc, int64_t M, int64_t N, int K, const void* Aq, const void* Bq,
                             const float* inv_sa, const float* inv_sb, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_gemm_update<OP, ST>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, gemm_lds_bytes());
    if (attr) return attr;
    const int tm = (int)((M + TM - 1) / TM), tn = (int)((N + TN - 1) / TN);
    const int nt = tm * tn;
    const int per_xcd = (nt + 7) / 8;
    // vectorised C access needs 16-byte aligned columns
    const int vec_ok = ((ldc * (int64_t)sizeof(typename Store<ST>::T)) % 16 == 0 && (((uintptr_t)C) % 16) == 0) ? 1 : 0;
    k_gemm_update<OP, ST><<<8 * per_xcd, 256, gemm_lds_bytes(), s>>>((typename Store<ST>::T*)C, ldc, M, N, K,
                                                                (const char*)Aq, (const char*)Bq, inv_sa, inv_sb,
                                                                tm, tn, per_xcd, vec_ok);
    return hipGetLastError();
}

hipError_t gemm_update(int update, int store, void* C, int64_t ldc, int64_t M, int64_t N, int K, const void* Aq,
                       const void* Bq, const float* inv_sa, const float* inv_sb, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if ((K * dtype_bytes(update)) % GBK) return hipErrorInvalidValue;
#define GCASE(U, S) if (update == U && store == S) return gemm_typed<U, S>(C, ldc, M, N, K, Aq, Bq, inv_sa, inv_sb, s)
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

}  // namespace mxp
