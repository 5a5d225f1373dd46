// gemm.hip -- the Schur-complement update of the blocked LU on the matrix
// cores (paper: "Algorithmic Framework", Figure 1: A22 <- A22 - A21 A11^-1 A12
// with 16-bit (here also 8-bit) inputs and 32-bit accumulation).
//
//   C (M x N, storage format, column-major, ldc)
//     <- C - diag(inv_sa) (Aq Bq^T) diag(inv_sb)
//   Aq: M x K operand (K-major rows), Bq: N x K operand (K-major rows),
//   inv_sa / inv_sb: one power-of-two factor per 32 rows / 32 columns.
//
// The accumulator starts at -C * (sa sb) (exact: powers of two), so the
// read of C is issued before the K loop and hidden behind it; the result is
// -acc * (inv_sa inv_sb), rounded once to the storage format.
//
// Tile 256 x 256, 512 threads = 8 waves in a 2 (M) x 4 (N) grid, each wave
// 128 x 64 = 4 x 2 blocks of 32 x 32 MFMA output.  K advances 128 bytes per
// stage through two LDS buffers (row pitch padded to 144 bytes so that the
// 16-byte fragment reads of 8 consecutive rows hit all 32 banks once).
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

constexpr int GT = 256;           // tile edge
constexpr int GBK = 128;          // K bytes per stage
constexpr int GPITCH = GBK + 16;  // LDS row pitch in bytes
constexpr int GSTAGE = GT * GPITCH;
constexpr int GGROUP = 8;         // tile rows per group in the tile order

template <int OP, int ST>
__global__ __launch_bounds__(512) void k_gemm_update(typename Store<ST>::T* C, int64_t ldc, int64_t M, int64_t N,
                                                     int K, const char* __restrict__ Aq, const char* __restrict__ Bq,
                                                     const float* __restrict__ inv_sa,
                                                     const float* __restrict__ inv_sb, int tiles_m, int tiles_n,
                                                     int per_xcd, int vec_ok) {
    typedef typename Store<ST>::T CT;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    char* sA = lds;                  // [2][GT][GPITCH]
    char* sB = lds + 2 * GSTAGE;     // [2][GT][GPITCH]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;     // 2 x 4 waves
    // tile order: XCD-contiguous ranges, grouped by GGROUP tile rows
    const int lin = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (lin >= tiles_m * tiles_n) return;
    const int group_size = GGROUP * tiles_n;
    const int grp = lin / group_size;
    const int first_m = grp * GGROUP;
    const int gm = (tiles_m - first_m) < GGROUP ? (tiles_m - first_m) : GGROUP;
    const int tm = first_m + (lin % group_size) % gm;
    const int tn = (lin % group_size) / gm;
    const int64_t row0 = (int64_t)tm * GT, col0 = (int64_t)tn * GT;
    constexpr int eb = sizeof(typename Operand<OP>::T);
    const int64_t Kbytes = (int64_t)K * eb;
    const char* gA = Aq + row0 * Kbytes;
    const char* gB = Bq + col0 * Kbytes;
    const int nst = (int)(Kbytes / GBK);
    const int lr = lane & 31, lh = lane >> 5;

    // ---- accumulator <- -C * (sa sb)
    f16v acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t rb = row0 + wm * 128 + a * 32;
        const float ia = inv_sa[rb / 32];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t cb = col0 + wn * 64 + b * 32;
            const float S = -1.0f / (ia * inv_sb[cb / 32]);
            const int64_t col = cb + lr;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t r = rb + 8 * g + 4 * lh;
                float v[4] = {0.f, 0.f, 0.f, 0.f};
                if (col < N) {
                    const CT* p = C + r + col * ldc;
                    if (vec_ok && r + 3 < M) Quad<ST>::load(p, v);
                    else
                        for (int q = 0; q < 4; ++q)
                            if (r + q < M) v[q] = Store<ST>::load(p, q);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[a][b][g * 4 + q] = v[q] * S;
            }
        }
    }

    // each thread moves 4 16-byte chunks of A and 4 of B per stage
    i4v ra[4], rb[4];
    auto gload = [&](int st) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int ch = tid + q * 512;          // 0..2047
            int r = ch >> 3, cb = (ch & 7) * 16;
            ra[q] = *(const i4v*)(gA + (int64_t)r * Kbytes + (int64_t)st * GBK + cb);
            rb[q] = *(const i4v*)(gB + (int64_t)r * Kbytes + (int64_t)st * GBK + cb);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int ch = tid + q * 512;
            int r = ch >> 3, cb = (ch & 7) * 16;
            *(i4v*)(sA + buf * GSTAGE + r * GPITCH + cb) = ra[q];
            *(i4v*)(sB + buf * GSTAGE + r * GPITCH + cb) = rb[q];
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    constexpr int KB = Mfma<OP>::KB;
    const int half = lh * (KB / 2);
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) gload(st + 1);
        const char* a_base = sA + buf * GSTAGE + (wm * 128 + lr) * GPITCH + half;
        const char* b_base = sB + buf * GSTAGE + (wn * 64 + lr) * GPITCH + half;
#pragma unroll(OP == F8 ? 1 : GBK / KB)
        for (int ks = 0; ks < GBK / KB; ++ks) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = Mfma<OP>::run(a_base + a * 32 * GPITCH + ks * KB, b_base + b * 32 * GPITCH + ks * KB,
                                              acc[a][b]);
        }
        if (st + 1 < nst) sstore(buf ^ 1);
        __syncthreads();
    }

    // ---- C <- -acc * (inv_sa inv_sb); lane holds column lr, rows 8g + 4 lh + q of each block
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t rb = row0 + wm * 128 + a * 32;
        const float ia = inv_sa[rb / 32];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t cb = col0 + wn * 64 + b * 32;
            const float d = -(ia * inv_sb[cb / 32]);
            const int64_t col = cb + lr;
            if (col >= N) continue;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int64_t r = rb + 8 * g + 4 * lh;
                float v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = acc[a][b][g * 4 + q] * d;
                CT* p = C + r + col * ldc;
                if (vec_ok && r + 3 < M) Quad<ST>::store(p, v);
                else
                    for (int q = 0; q < 4; ++q)
                        if (r + q < M) p[q] = Store<ST>::from_f32(v[q]);
            }
        }
    }
}

template <int OP, int ST>
static hipError_t gemm_typed(void* C, int64_t ldc, int64_t M, int64_t N, int K, const void* Aq, const void* Bq,
                             const float* inv_sa, const float* inv_sb, hipStream_t s) {
    static bool attr_done = false;
    hipError_t e;
    if (!attr_done) {
        if ((e = hipFuncSetAttribute((const void*)k_gemm_update<OP, ST>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     4 * GSTAGE)))
            return e;
        attr_done = true;
    }
    const int tm = (int)((M + GT - 1) / GT), tn = (int)((N + GT - 1) / GT);
    const int nt = tm * tn;
    const int per_xcd = (nt + 7) / 8;
    const int vec_ok = ((ldc % 4) == 0 && (((uintptr_t)C) % 16) == 0) ? 1 : 0;
    k_gemm_update<OP, ST><<<8 * per_xcd, 512, 4 * GSTAGE, s>>>((typename Store<ST>::T*)C, ldc, M, N, K,
                                                              (const char*)Aq, (const char*)Bq, inv_sa, inv_sb, tm,
                                                              tn, per_xcd, vec_ok);
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
