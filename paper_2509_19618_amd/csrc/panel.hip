// panel.hip -- the strip solves of a block step as products with the
// diagonal block's inverses (paper: "Algorithmic Framework", Figure 1: the
// Schur complement written A22 - A21 A11^-1 A12, the triangular solves in
// 32-bit arithmetic, a custom mixed-precision scheme permitted).
//
// With A11 = L11 U11 factored in FP32 and the full FP32 inverses of L11 and
// U11 formed, the strips are
//   L21 = A21 U11^-1      (rows of the block column below the diagonal block)
//   U12 = L11^-1 A12      (columns of the block row right of it),
// products without a dependency chain.  They run on the 16-bit matrix cores
// of the storage format: the stored panel is exact in that format, and each
// inverse is split into NS parts of it whose sum carries about 22 (FP16:
// hi + lo under a power-of-two scale per line, which keeps the parts in the
// normal range) or 24 (BF16: hi + mid + lo) significant bits, so that with
// FP32 accumulation the strips keep FP32 quality.  The epilogue is the one of
// the substitution it replaces: a power-of-two scale per 32-row (column)
// strip from the strip's largest magnitude, the operand of the trailing
// update rounded under it, the stored strip written back.
#include "common.hpp"
#include "kernels.hpp"

namespace mxp {

typedef _Float16 ph8 __attribute__((ext_vector_type(8)));
typedef __bf16 pb8 __attribute__((ext_vector_type(8)));
typedef unsigned short pu8 __attribute__((ext_vector_type(8)));
typedef float pf16 __attribute__((ext_vector_type(16)));
typedef int pi4 __attribute__((ext_vector_type(4)));

template <int ST> struct Split;
template <> struct Split<F16> {
    static constexpr int NS = 2;
    static MXP_DEV unsigned short bits(float v) { half_t h = (half_t)v; return __builtin_bit_cast(unsigned short, h); }
    static MXP_DEV float val(unsigned short b) { return (float)__builtin_bit_cast(half_t, b); }
    static MXP_DEV pf16 mma(pu8 a, pu8 b, pf16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(ph8, a), __builtin_bit_cast(ph8, b), c, 0, 0, 0);
    }
};
template <> struct Split<BF16> {
    static constexpr int NS = 3;
    static MXP_DEV unsigned short bits(float v) { return f32_to_bf16_bits(v); }
    static MXP_DEV float val(unsigned short b) { return bf16_bits_to_f32(b); }
    static MXP_DEV pf16 mma(pu8 a, pu8 b, pf16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pb8, a), __builtin_bit_cast(pb8, b), c, 0, 0, 0);
    }
};

bool panel_path(int store) { return store == F16 || store == BF16; }

// Fragment order of the parts: the B fragment of output column block J at
// k-step ks (K = 16 ks .. 16 ks + 15) is 64 lanes x 8 halves, contiguous
// (1 KB), lane l = 32 (K / 8 % 2) + (line % 32) holding K = 16 ks + 8 (l / 32)
// .. +7 of line 32 J + l % 32.  Offset (halves) of the 8-run starting at K
// (a multiple of 8) of a line:
__host__ __device__ inline int64_t frag_off(int nb, int line, int kk) {
    const int J = line >> 5, lr = line & 31, ks = kk >> 4, lh = (kk >> 3) & 1;
    return ((int64_t)(J * (nb >> 4) + ks) * 64 + lh * 32 + lr) * 8;
}

// ------------------------------------------------------------------ split of the inverses
// Work-group w of a block: 16 columns of U11^-1 (w < nb/16) or 16 rows of
// L11^-1.  A line x (a column c of U11^-1, a row j of L11^-1: the K-run of
// one output column of the strip products) gets sigma = 2^-ceil(log2
// max|x|) and parts p_0 = rnd(sigma x), p_s = rnd(sigma x - sum_{t<s} p_t);
// each difference is exact in FP32.  Stored: part s of line l in fragment
// order (frag_off), zero for kk > l (the inverses are triangular), and
// 1/sigma per line.
template <int ST>
__global__ __launch_bounds__(256) void k_inv_split(const PanelGroup grp) {
    extern __shared__ float sm[];
    int d = 0;
    while ((int)blockIdx.x >= grp.g[d].wg_split) ++d;
    const PanelOne& G = grp.g[d];
    const int w0 = (int)blockIdx.x - (d > 0 ? grp.g[d - 1].wg_split : 0);
    const int nb = G.nb, P = nb + 1, nl = nb / 16;
    const bool uside = w0 < nl;
    const int l0 = 16 * (uside ? w0 : w0 - nl);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ldi = G.ldi;
    // eight loads in flight per lane; an index past the 16 lines reads
    // element 0 of the first line again (not stored)
    const int tot = 16 * nb;
    for (int e0 = 0; e0 < tot; e0 += 2048) {
        float x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = e0 + tid + 256 * i < tot ? e0 + tid + 256 * i : 0;
            x[i] = uside ? G.Ui[(e % nb) + (int64_t)(l0 + e / nb) * ldi] : G.Li[(l0 + (e & 15)) + (int64_t)(e >> 4) * ldi];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = e0 + tid + 256 * i;
            if (e < tot) {
                if (uside) sm[(e / nb) * P + e % nb] = x[i];
                else sm[(e & 15) * P + (e >> 4)] = x[i];
            }
        }
    }
    __syncthreads();
    unsigned short* parts = (unsigned short*)(uside ? G.ub : G.lb);
    float* rs = uside ? G.ubs : G.lbs;
    float* scl = sm + 16 * P;                         // the 16 line scales
    for (int li = 0; li < 4; ++li) {
        const int line = wave * 4 + li;
        float m = 0.0f;
        for (int kk = lane; kk <= l0 + line; kk += 64) m = fmaxf(m, fabsf(sm[line * P + kk]));
        m = warp_maxf(m);
        const float sc = pow2_scale(m, 0);
        if (lane == 0) {
            rs[l0 + line] = 1.0f / sc;
            scl[line] = sc;
        }
    }
    __syncthreads();
    // a lane: 8 consecutive K of one line (16 bytes per part); lanes run over
    // the lines first, so that a wave's stores fill whole fragments' runs
    const int64_t plane = (int64_t)nb * nb;
    for (int e = tid; e < 2 * nb; e += 256) {
        const int line = e & 15, c8 = e >> 4;             // chunk c8: K = 8 c8 .. 8 c8 + 7
        const int gl = l0 + line;
        const float sc = scl[line];
        pu8 o[Split<ST>::NS];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int kk = 8 * c8 + t;
            // past the triangle (K beyond the line's own index) the parts are zero
            float r = kk <= gl ? sm[line * P + kk] * sc : 0.0f;
#pragma unroll
            for (int s2 = 0; s2 < Split<ST>::NS; ++s2) {
                const unsigned short bits = Split<ST>::bits(r);
                o[s2][t] = bits;
                r -= Split<ST>::val(bits);
            }
        }
        const int64_t off = frag_off(nb, gl, 8 * c8);
#pragma unroll
        for (int s2 = 0; s2 < Split<ST>::NS; ++s2) *(pu8*)(parts + s2 * plane + off) = o[s2];
    }
}

hipError_t panel_split(int store, const PanelGroup& grp, int wg, int nbmax, hipStream_t s) {
    const size_t smem = (size_t)16 * (nbmax + 2) * 4;
    static const hipError_t attr = []() {
        hipError_t e;
        if ((e = hipFuncSetAttribute((const void*)k_inv_split<F16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     16 * 1026 * 4))) return e;
        return hipFuncSetAttribute((const void*)k_inv_split<BF16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   16 * 1026 * 4);
    }();
    if (attr) return attr;
    if (store == F16) k_inv_split<F16><<<wg, 256, smem, s>>>(grp);
    else if (store == BF16) k_inv_split<BF16><<<wg, 256, smem, s>>>(grp);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------ strip products
// One work-group: TR = 32 RB rows of L21 (work-groups [0, ntile)) or TR
// columns of U12 (the rest), all nb output columns.  The panel tile goes to
// LDS once: the rows of A21 as stored (column-major: K runs over the LDS
// rows, [kk][row]), the columns of A12 with K contiguous ([row][kk]).  The
// NW waves share the tile; wave v owns the 32-wide output column blocks
// J = v, v+NW, ... (at most four) and runs each over K in [0, 32 (J+1))
// only (the inverses are triangular).  The split parts stream from L2 into
// the B fragments (fragment order: one contiguous kilobyte per fragment),
// several k-steps ahead of their use.  MFMA 32x32x16: lane l holds A row l%32 / B column l%32
// with K = 8 (l/32) .. +8; result register q of lane l is row 8(q/4) +
// 4(l/32) + q%4, column l%32.
// Tile shapes: FP16 storage and nb <= 512: 64 rows, four waves; otherwise
// (nb > 512, or BF16 with its three parts, whose fragments would not fit in
// registers beside two row blocks): 32 rows, eight waves.
int panel_rows(int store, int nb) { return (store == F16 && nb <= 512) ? 64 : 32; }
__host__ __device__ static inline size_t panel_smem(int nb, int TR) {
    size_t a = (size_t)nb * (TR + 8) * 2;                 // L tile / L storage stage
    size_t b = (size_t)TR * (nb + 8) * 2;                 // U tile / U storage stage
    size_t c = (size_t)TR * (nb + 16) * 2;                // operand stage (at most 2 bytes an element)
    size_t m = a > b ? a : b;
    m = m > c ? m : c;
    return m + 128;                                      // + the strip maxima, and the slack of the
                                                         // A fragment read ahead of a block's last k-step
}

template <int ST, int OP, int RB, int NW>
__global__ __launch_bounds__(64 * NW, 8 / NW) void k_trsm_inv(const PanelGroup grp) {
    typedef typename Store<ST>::T STT;
    typedef typename Operand<OP>::T OPT;
    constexpr int NS = Split<ST>::NS;
    constexpr int TR = 32 * RB, NT = 64 * NW, CBM = 4;
    constexpr int PL = TR + 8;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    int d = 0;
    while ((int)blockIdx.x >= grp.g[d].wg_trsm) ++d;
    const PanelOne& G = grp.g[d];
    const int w0 = (int)blockIdx.x - (d > 0 ? grp.g[d - 1].wg_trsm : 0);
    const bool lside = w0 < G.ntile;                      // work-group uniform
    const int tile = lside ? w0 : w0 - G.ntile;
    const int nb = G.nb, PU = nb + 8;
    const int64_t n = G.n, k = G.k, lda = G.lda;
    STT* A = (STT*)G.A;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 31, lh = lane >> 5;
    const int64_t base = k + nb + (int64_t)TR * tile;    // first row (L side) / column (U side) of the tile
    const int64_t nvl = n - base;
    const int nv = (int)(nvl > TR ? TR : (nvl < 0 ? 0 : nvl));
    unsigned short* sl = (unsigned short*)lds;
    float* red = (float*)(lds + panel_smem(nb, TR) - 64);
    const bool al = (lda & 7) == 0 && ((uintptr_t)A & 15) == 0;

    // ---- the panel tile into LDS as [row][kk] (row: a row of A21 or a
    // column of A12; pitch nb + 8 halves), the 16-byte chunk c of row r
    // stored at chunk c ^ ((r >> 4) & 3): the MFMA fragment reads (16 bytes,
    // rows over the lanes) and the transposing 2-byte writes of the A21 rows
    // spread over the 64 banks.  Every load of a batch is in flight at once;
    // an index past the range reads a valid element, not stored.
    auto tix = [&](int r, int kk) { return r * PU + ((((kk >> 3) ^ (r >> 4)) & 3) | ((kk >> 3) & ~3)) * 8 + (kk & 7); };
    if (lside) {
        if (al && nv == TR) {
            // a lane: 8 consecutive rows of one column (16 bytes), written as 8 halves
            constexpr int RG = TR / 8;
            const int tot = nb * RG;
            for (int e0 = 0; e0 < tot; e0 += 8 * NT) {
                pu8 x[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int e = e0 + tid + NT * i;
                    const int rg = e % RG, c = e < tot ? e / RG : 0;
                    x[i] = *(const pu8*)(A + (base + 8 * rg) + (k + c) * lda);
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int e = e0 + tid + NT * i;
                    const int rg = e % RG, c = e / RG;
                    if (e < tot)
#pragma unroll
                        for (int q = 0; q < 8; ++q) sl[tix(8 * rg + q, c)] = x[i][q];
                }
            }
        } else {
            for (int e = tid; e < nb * TR; e += NT) {
                const int r = e % TR, c = e / TR;
                sl[tix(r, c)] = r < nv ? *(const unsigned short*)(A + (base + r) + (k + c) * lda) : (unsigned short)0;
            }
        }
    } else {
        if (al) {
            // a lane: 8 consecutive K of one column (16 bytes); a column past
            // the matrix reads column k + nb
            const int KG = nb / 8;
            const int tot = TR * KG;
            for (int e0 = 0; e0 < tot; e0 += 8 * NT) {
                pi4 x[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int e = e0 + tid + NT * i;
                    const int kg = e % KG, r = e / KG;
                    const int64_t col = (e < tot && r < nv) ? base + r : k + nb;
                    x[i] = *(const pi4*)(A + (k + 8 * kg) + col * lda);
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int e = e0 + tid + NT * i;
                    const int kg = e % KG, r = e / KG;
                    if (e < tot) {
                        pi4 v = x[i];
                        if (r >= nv) v = pi4{0, 0, 0, 0};
                        *(pi4*)(sl + tix(r, 8 * kg)) = v;
                    }
                }
            }
        } else {
            for (int e = tid; e < nb * TR; e += NT) {
                const int kk = e % nb, r = e / nb;
                sl[tix(r, kk)] = r < nv ? *(const unsigned short*)(A + (k + kk) + (base + r) * lda) : (unsigned short)0;
            }
        }
    }
    __syncthreads();

    // ---- the products: per column block, the K loop with the B fragments of
    // the next PD k-steps in flight (a ring of registers).  A block's K range
    // is rounded up to a multiple of PD (at most nb): the parts are exactly
    // zero past the triangle, so the extra steps add zeros and the loop body
    // runs without branches (its B loads past the range re-read the last
    // step; the A fragment read ahead of the last step is not used)
    constexpr int PD = 4;
    const int nJ = nb / 32, nks_max = nb / 16;
    const int ncb = (nJ - wave + NW - 1) / NW;            // this wave's column blocks (0: idle)
    const unsigned short* parts = (const unsigned short*)(lside ? G.ub : G.lb);
    const int64_t plane = (int64_t)nb * nb;
    pf16 acc[RB][CBM];
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < CBM; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    const int boff = 8 * lane;                           // this lane's 16 bytes of a fragment
    // A fragment of row block rb at k-step ks: chunk 2 ks + lh of row 32 rb + lr;
    // the swizzle touches the low two chunk bits only, so the address is a
    // per-lane base for the parity of ks plus 32 halves per pair of k-steps
    const unsigned short* abase[RB][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int par = 0; par < 2; ++par) abase[rb][par] = sl + tix(32 * rb + lr, 16 * par + 8 * lh);
    auto lda_frag = [&](pu8 (&af)[RB], int ks, int par) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) af[rb] = *(const pu8*)(abase[rb][par] + 32 * (ks >> 1));
    };
#pragma unroll
    for (int cb = 0; cb < CBM; ++cb) {
        if (cb < ncb) {                                   // wave-uniform
            const int J = wave + NW * cb;
            int nk = (2 * (J + 1) + PD - 1) / PD * PD;
            nk = nk < nks_max ? nk : nks_max;
            const unsigned short* bp = parts + (int64_t)J * (nb >> 4) * 512 + boff;
            auto ldb = [&](pu8 (&bf)[NS], int ks) {
                ks = ks < nk ? ks : nk - 1;
#pragma unroll
                for (int s2 = 0; s2 < NS; ++s2) bf[s2] = *(const pu8*)(bp + s2 * plane + 512 * ks);
            };
            pu8 ring[PD][NS], af[RB], an[RB];
#pragma unroll
            for (int i = 0; i < PD; ++i) {
                ldb(ring[i], i);
                __builtin_amdgcn_sched_barrier(0);        // issued in the order of use
            }
            lda_frag(af, 0, 0);
            for (int k0 = 0; k0 < nk; k0 += PD) {
#pragma unroll
                for (int i = 0; i < PD; ++i) {
                    const int ks = k0 + i;                // k0 is a multiple of PD: the parity of ks is i's
                    lda_frag(an, ks + 1, (i + 1) & 1);
#pragma unroll
                    for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb)
                            acc[rb][cb] = Split<ST>::mma(af[rb], ring[i][s2], acc[rb][cb]);
                    ldb(ring[i], ks + PD);
                    // keep the loads where they are issued: scheduled next
                    // to their uses they would wait out their whole latency
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) af[rb] = an[rb];
                }
            }
        }
    }

    // ---- epilogue: undo the line scales, strip maxima, scales
    const float* rsc = lside ? G.ubs : G.lbs;
    float mx[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) mx[rb] = 0.0f;
#pragma unroll
    for (int cb = 0; cb < CBM; ++cb) {
        if (cb < ncb) {
            const float f = rsc[32 * (wave + NW * cb) + lr];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    acc[rb][cb][r] *= f;
                    mx[rb] = fmaxf(mx[rb], fabsf(acc[rb][cb][r]));
                }
        }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const float v = warp_maxf(mx[rb]);
        if (lane == 0) red[wave * RB + rb] = v;
    }
    __syncthreads();                                      // maxima visible; the panel tile no longer read
    float s_op[RB], s_st[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        float amax = 0.0f;
#pragma unroll
        for (int v = 0; v < NW; ++v) amax = fmaxf(amax, red[v * RB + rb]);
        s_op[rb] = Operand<OP>::scaled ? pow2_scale(amax, Operand<OP>::scale_exp) : 1.0f;
        s_st[rb] = (lside && Store<ST>::scaled) ? pow2_scale(amax, Store<ST>::scale_exp) : 1.0f;
    }
    const int strip0 = RB * tile;                         // first 32-wide strip of the tile in this block step
    if (tid < RB) {
        if (lside) {
            G.inv_sa[strip0 + tid] = 1.0f / s_op[tid];
            if (32 * tid < nv) G.lsc_blk[(base + 32 * tid) / 32] = s_st[tid];
        } else {
            G.inv_sb[strip0 + tid] = 1.0f / s_op[tid];
        }
    }

    // ---- the operand rows (K-major: nb contiguous values per row) through LDS
    {
        constexpr int OB = (int)sizeof(OPT);
        const int PO = nb + 16;                           // elements; PO * OB a multiple of 16 bytes
        OPT* so = (OPT*)lds;
#pragma unroll
        for (int cb = 0; cb < CBM; ++cb)
            if (cb < ncb)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int row = 32 * rb + 8 * (q >> 2) + 4 * lh + (q & 3);
                        so[row * PO + 32 * (wave + NW * cb) + lr] = Operand<OP>::from_f32(acc[rb][cb][q] * s_op[rb]);
                    }
        __syncthreads();
        char* dst = (char*)(lside ? G.Lq : G.Uq) + (int64_t)TR * tile * nb * OB;
        const int cpr = nb * OB / 16;                     // 16-byte chunks per row
        for (int e = tid; e < TR * cpr; e += NT) {
            const int row = e / cpr, ch = e - row * cpr;
            *(pi4*)(dst + ((int64_t)row * nb * OB + ch * 16)) = *(const pi4*)((const char*)so + row * PO * OB + ch * 16);
        }
        __syncthreads();
    }

    // ---- the stored strip
    if (lside) {
        // L21 (scaled by s_st), column-major: stage [col][row]
#pragma unroll
        for (int cb = 0; cb < CBM; ++cb)
            if (cb < ncb)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int row = 32 * rb + 8 * (q >> 2) + 4 * lh + (q & 3);
                        const STT v = Store<ST>::from_f32(acc[rb][cb][q] * s_st[rb]);
                        sl[(32 * (wave + NW * cb) + lr) * PL + row] = __builtin_bit_cast(unsigned short, v);
                    }
        __syncthreads();
        if (al && nv == TR) {
            constexpr int RG = TR / 8;
            for (int e = tid; e < nb * RG; e += NT) {
                const int rg = e % RG, c = e / RG;
                *(pi4*)(A + (base + 8 * rg) + (k + c) * lda) = *(const pi4*)(sl + c * PL + 8 * rg);
            }
        } else {
            for (int e = tid; e < nb * TR; e += NT) {
                const int r = e % TR, c = e / TR;
                if (r < nv) *(unsigned short*)(A + (base + r) + (k + c) * lda) = sl[c * PL + r];
            }
        }
    } else {
        // U12 (unscaled): row r of the tile is column base + r, K contiguous: stage [row][kk]
#pragma unroll
        for (int cb = 0; cb < CBM; ++cb)
            if (cb < ncb)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int row = 32 * rb + 8 * (q >> 2) + 4 * lh + (q & 3);
                        const STT v = Store<ST>::from_f32(acc[rb][cb][q]);
                        sl[row * PU + 32 * (wave + NW * cb) + lr] = __builtin_bit_cast(unsigned short, v);
                    }
        __syncthreads();
        if (al) {
            const int KG = nb / 8;
            for (int e = tid; e < TR * KG; e += NT) {
                const int kg = e % KG, r = e / KG;
                if (r < nv) *(pi4*)(A + (k + 8 * kg) + (base + r) * lda) = *(const pi4*)(sl + r * PU + 8 * kg);
            }
        } else {
            for (int e = tid; e < nb * TR; e += NT) {
                const int kk = e % nb, r = e / nb;
                if (r < nv) *(unsigned short*)(A + (k + kk) + (base + r) * lda) = sl[r * PU + kk];
            }
        }
    }
}

template <int ST, int OP>
static hipError_t trsm_launch(const PanelGroup& grp, int wg, int nbmax, hipStream_t s) {
    static const hipError_t attr = []() {
        hipError_t e;
        if constexpr (ST == F16)
            if ((e = hipFuncSetAttribute((const void*)k_trsm_inv<ST, OP, 2, 4>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)panel_smem(512, 64))))
                return e;
        return hipFuncSetAttribute((const void*)k_trsm_inv<ST, OP, 1, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)panel_smem(1024, 32));
    }();
    if (attr) return attr;
    if constexpr (ST == F16)
        if (panel_rows(ST, nbmax) == 64) {
            k_trsm_inv<ST, OP, 2, 4><<<wg, 256, panel_smem(nbmax, 64), s>>>(grp);
            return hipGetLastError();
        }
    k_trsm_inv<ST, OP, 1, 8><<<wg, 512, panel_smem(nbmax, 32), s>>>(grp);
    return hipGetLastError();
}

hipError_t panel_trsm(int store, int update, const PanelGroup& grp, int wg, int nbmax, hipStream_t s) {
    if (store == F16 && update == F16) return trsm_launch<F16, F16>(grp, wg, nbmax, s);
    if (store == BF16 && update == BF16) return trsm_launch<BF16, BF16>(grp, wg, nbmax, s);
    if (store == F16 && update == F8) return trsm_launch<F16, F8>(grp, wg, nbmax, s);
    if (store == BF16 && update == F8) return trsm_launch<BF16, F8>(grp, wg, nbmax, s);
    return hipErrorInvalidValue;
}

}  // namespace mxp
