// kernels.hpp -- host-side launchers of the libmxp kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mxp {

// ---- generation / residual (gen.hip)
hipError_t fill_u64(void* p, int64_t count, uint64_t v, hipStream_t s);
// kind: 0 diagonally dominant, 1 diagonal gamma sqrt(n) (shift = gamma sqrt(n)),
// 2 uniform in [-1, 1) without diagonal change
hipError_t generate(int64_t n, int64_t nrhs, uint64_t seed, int kind, double shift, int store, void* A, int64_t lda,
                    double* B, int64_t ldb, double* diag, double* row_l1, double* a_inf, hipStream_t s);
// value of one unit of a draw offset k - 2^31 in the matrix of a kind
double gen_offscale(int kind);
int64_t regen_chunk_cols(int64_t n);
size_t regen_partial_bytes(int64_t n, int nr);
hipError_t regen_matvec(int64_t n, uint64_t seed, int kind, const double* diag, const double* X, int64_t ldx, int nr,
                        const double* B, int64_t ldb, double* R, int64_t ldr, double* P, hipStream_t s);
int eta_blocks(int64_t n);
// the library's file-scope device scratch array (device address on the
// current device, looked up once per device) and its size
hipError_t static_scratch(void** out);
size_t static_scratch_bytes();
// eta_out[4 q] = HPL scaled residual of right-hand side q (q < nr), [4 q + 1]
// ||x_q||_inf, [4 q + 2] ||r_q||_inf; part: eta_blocks(n) * 3 * nr doubles
hipError_t hpl_eta_dev(int64_t n, int nr, const double* r, int64_t ldr, const double* x, int64_t ldx,
                       const double* b, int64_t ldb, const double* a_inf, double* part, double* eta_out,
                       hipStream_t s);

// ---- factorisation (lu.hip)
struct FactorPlan {
    int64_t n, nb, lda;
    int update, store;
    void* A;         // the matrix, overwritten by L\U
    // aux (persistent)
    float* T;        // nblk x nb x nb: FP32 L11\U11 of every diagonal block
    float* Trm;      // nblk x nb x nb: the same, row-major
    float* linv;     // nblk x (nb/64) x 64 x 64: inverses of the unit-lower 64x64 diagonal sub-blocks
    float* uinv;     // same for U
    float* lsc;      // nblk x ceil(n/32): power-of-two scale of every stored 32-row strip of L21
    double* rowscale;  // n
    float* linv_full;  // ngrp x D x D (D = prec_block(nb)): inverses of the unit-lower parts of the
                       // preconditioner's diagonal blocks (FP32, column-major, ld D)
    float* uinv_full;  // the same for the upper parts
    // work (scratch)
    int64_t op_rows; // rows of one operand set (operand_rows(n))
    void* Lq;        // 4 sets of op_rows x nb operands (K-major)
    void* Uq;        // 4 sets of op_rows x nb operands (K-major)
    float* inv_sa;   // 4 sets of op_rows/32
    float* inv_sb;   // 4 sets of op_rows/32
    float* pairw;    // ceil(n / 2nb) x nb x nb: scratch of the pair inverses (D = 2 nb only)
    void* binv;      // 2 x 3 x nb x nb 16-bit parts of the current block's inverses (U11^-1, L11^-1)
    float* binv_sc;  // 2 x nb reciprocal line scales of those parts
    unsigned long long* info;  // 1
    int* dsync;      // nblk x diag_sync_words(): phase counters of the diagonal-block LUs (zeroed per factorisation)
    int gemm_tile = 0;  // work-group tile of the trailing update (GEMM_TILE_*)
};

struct AuxLayout {
    size_t T, Trm, linv, uinv, lsc, rowscale, linv_full, uinv_full, total;
};
struct WorkLayout {
    size_t Lq, Uq, inv_sa, inv_sb, info, dsync, pairw, binv, binv_sc, total;
};
AuxLayout aux_layout(int64_t n, int64_t nb);
// diagonal-block size of the preconditioner's substitution: pairs of factor
// blocks for nb <= 512 (one hand-over between work-groups per pair), the
// factor blocks otherwise
#ifndef MXP_PREC_PAIRS
#define MXP_PREC_PAIRS 1
#endif
__host__ __device__ inline int64_t prec_block(int64_t nb) { return (MXP_PREC_PAIRS && nb <= 512) ? 2 * nb : nb; }
int64_t operand_rows(int64_t n);
WorkLayout work_layout(int64_t n, int64_t nb, int update);
int dtype_bytes(int dt);

// C (M x N, storage) <- C - diag(inv_sa) Aq Bq^T diag(inv_sb); Aq/Bq rows padded to 256.
// With a second segment (K2 > 0: the operands of the next block step, with
// their own factors) the update of both steps is accumulated in one pass:
// C <- C - [diag(inv_sa) Aq Bq^T diag(inv_sb) + diag(inv_sa2) Aq2 Bq2^T diag(inv_sb2)],
// rounded to the storage format once.
// tile: the work-group tile of the update kernel (256 x 128 or 128 x 128).
enum { GEMM_TILE_256 = 0, GEMM_TILE_128 = 1 };
constexpr int GEMM_GROUP_MAX = 8;   // factorisations served by one grouped launch
constexpr int GEMM_DESC_MAX = 16;   // update descriptors of one launch
struct GemmCall {
    void* C;
    int64_t ldc, M, N;
    int K;
    const void* Aq;
    const void* Bq;
    const float* inv_sa;
    const float* inv_sb;
    int K2 = 0;
    const void* Aq2 = nullptr;
    const void* Bq2 = nullptr;
    const float* inv_sa2 = nullptr;
    const float* inv_sb2 = nullptr;
};
int gemm_tile_rows(int tile);
hipError_t gemm_update(int update, int store, void* C, int64_t ldc, int64_t M, int64_t N, int K, const void* Aq,
                       const void* Bq, const float* inv_sa, const float* inv_sb, hipStream_t s,
                       int tile = GEMM_TILE_256);
// up to GEMM_DESC_MAX independent updates (same formats and tile) in one launch
hipError_t gemm_group(int update, int store, int tile, const GemmCall* calls, int count, hipStream_t s);
// FP32 LU of the diagonal block A[k:k+kb, k:k+kb] (padded to kbp, a multiple
// of 64, with the identity) by a few cooperating work-groups: T/Trm (ld ldt)
// get L\U column- and row-major, linv/uinv the 64x64 sub-block inverses, A
// the factored block.  sync: diag_sync_words() zeroed ints for this call.  A
// zero / non-finite pivot sets *info (atomic min) to its 1-based column; an
// expired wait sets it to 2^62.
size_t diag_sync_words();
struct DiagCall {
    void* A;
    int64_t lda, k;
    int kb, kbp, ldt;
    float *T, *Trm, *linv, *uinv;
    int* sync;
    unsigned long long* info;
};
// Strip solves through the diagonal block's inverses (16-bit storage,
// panel.hip): per block step, (1) block_inverses: the full FP32 inverses of
// L11 and U11 (the preconditioner's diagonal blocks, formed once here);
// (2) panel_split: each inverse split into 16-bit parts of the storage format
// under a power-of-two scale per line; (3) panel_trsm: L21 = A21 U11^-1 and
// U12 = L11^-1 A12 on the 16-bit matrix cores with FP32 accumulation, fused
// with the rounding to the update format under a power-of-two strip scale.
// One launch of each serves a group of factorisations: every kernel finds
// its descriptor by its work-group number (cumulative ends per kernel).
struct PanelOne {
    void* A;
    int64_t lda, n, k, ldi;
    int nb, kbp, ntile, pad;                 // ntile: output tiles of panel_rows(launch nb) per side
    int wg_inv, wg_split, wg_trsm, pad2;
    const float *T, *Trm, *linv, *uinv;      // the block's FP32 factor and 64x64 sub-block inverses
    float *Li, *Ui;                          // the block's FP32 inverses (column-major, ld ldi)
    void *lb, *ub;                           // their 16-bit parts
    float *lbs, *ubs;                        // reciprocal line scales of the parts
    void* Lq;
    float* inv_sa;
    float* lsc_blk;
    void* Uq;
    float* inv_sb;
};
struct PanelGroup {
    PanelOne g[GEMM_GROUP_MAX];
    int count;
};
bool panel_path(int store);                  // FP16 and BF16 storage
int panel_rows(int store, int nb);           // rows (columns) of an output tile of panel_trsm
hipError_t block_inverses(const PanelGroup& grp, int wg, int nbmax, hipStream_t s);
hipError_t panel_split(int store, const PanelGroup& grp, int wg, int nbmax, hipStream_t s);
hipError_t panel_trsm(int store, int update, const PanelGroup& grp, int wg, int nbmax, hipStream_t s);
// the diagonal-block LUs of up to GEMM_GROUP_MAX factorisations in one launch
hipError_t diag_lu_group(int store, const DiagCall* calls, int count, hipStream_t s);
hipError_t diag_lu(int store, void* A, int64_t lda, int64_t k, int kb, int kbp, float* T, float* Trm, int ldt,
                   float* linv, float* uinv, int* sync, unsigned long long* info, hipStream_t s);
hipError_t row_equilibrate(const FactorPlan& p, const double* diag, hipStream_t s);
// Side stream and events of the look-ahead (default stream priority): the
// side stream carries the chain of a factorisation (diagonal-block update,
// LU, strip TRSMs, the next block column and row by one step); the events
// order it against the caller's stream, which runs the merged updates
// (ev_upd: the last part of a pair's update, ev_cross / ev_next: its first
// two parts, ev_panel: the panels of the next pair).  A factorisation uses
// the caller's context, or one from a per-device pool if la is NULL.
struct Lookahead {
    hipStream_t side = nullptr;
    hipEvent_t ev_upd = nullptr, ev_cross = nullptr, ev_next = nullptr, ev_panel = nullptr;
};
hipError_t lookahead_create(Lookahead* la);
void lookahead_destroy(Lookahead* la);
hipError_t factor_run(const FactorPlan& p, hipStream_t s, Lookahead* la = nullptr);
// up to GEMM_GROUP_MAX factorisations (same formats, any sizes) in lockstep on
// one stream: per block step one launch each of the diagonal-block LUs and
// the strip TRSMs of all of them, and per pair of steps one launch of the
// next block column / row updates and one of the merged updates (no
// look-ahead; the arithmetic of factor_run)
hipError_t factor_group(const FactorPlan* plans, int count, hipStream_t s);
// mxp_factor with an explicit look-ahead context (api.hip)
int factor_with(int64_t n, int64_t nb, int update, int store, int scaling, const double* diag, void* A, int64_t lda,
                void* aux, void* work, size_t work_bytes, int64_t* info, hipStream_t s, Lookahead* la);

// ---- FP64 LU with or without partial pivoting (lu64.hip)
int lu64_block(int64_t n);
size_t lu64_work_bytes(int64_t n);
int* lu64_err_word(void* work, int64_t n);
hipError_t lu64_factor(int64_t n, double* A, int64_t lda, int64_t* ipiv, void* work, unsigned long long* info_dev,
                       int use_rocblas, hipStream_t s);
hipError_t lu64_solve(int64_t n, const double* A, int64_t lda, const int64_t* ipiv, double* X, int64_t ldx, int nr,
                      hipStream_t s);
hipError_t gemm64(double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                  int64_t N, int K, hipStream_t s);

// ---- preconditioner and GMRES pieces (solve.hip)
struct PrecPlan {
    int64_t n, nb, lda;
    int store;
    const void* A;      // L\U in storage format
    const float* T;     // aux pieces (see FactorPlan)
    const float* linv;
    const float* uinv;
    const float* lsc;
    const double* rowscale;
    const float* linv_full;
    const float* uinv_full;
};
// Z = U^-1 L^-1 S V for nr columns (V may alias Z); W: prec_work_bytes(n, nr)
// of scratch.  A wait of the substitution kernels that expires sets an error
// word in W (cleared by prec_err_reset, read by prec_err_read).
size_t prec_work_bytes(int64_t n, int nr);
hipError_t prec_apply(const PrecPlan& p, const double* V, int64_t ldv, double* Z, int64_t ldz, int nr, double* W,
                      hipStream_t s);
hipError_t prec_err_reset(double* W, int64_t n, int nr, hipStream_t s);
hipError_t prec_err_read(double* W, int64_t n, int nr, int* err, hipStream_t s);

// GMRES steps for nr right-hand sides in lockstep (solve.hip).  V holds the
// bases, v_{r,j} at V + (j nr + r) n; W the new vectors (n x nr); H, cs, sn,
// g, y per right-hand side with ldh = m + 1 (H: ldh x m each); part: 2 x nr x
// 256 partial sums; act[r]: right-hand side r takes part; sc: per-r scalars
// with stride sc_stride.
hipError_t gm_norms(int64_t n, int nr, const double* X, int64_t ldx, double* out, int out_stride, double* part,
                    const int* act, hipStream_t s);
hipError_t gm_start(int64_t n, int nr, const double* Z, const double* sc, int sc_stride, double* V, double* g,
                    int ldg, const int* act, hipStream_t s);
hipError_t gm_arnoldi(int64_t n, int nr, double* V, int k, double* W, double* part, double* H, int ldh,
                      const int* act, hipStream_t s);
hipError_t gm_givens(int nr, int k, double* H, int ldh, double* cs, double* sn, double* g, const double* sc,
                     int sc_stride, double tau, int* flag, const int* act, hipStream_t s);
hipError_t gm_update(int64_t n, int nr, const double* H, int ldh, const double* g, double* y, const int* kdim,
                     const double* V, double* X, int64_t ldx, hipStream_t s);
hipError_t set_i32(int* dst, int n, const int* src_dev, hipStream_t s);
int red_blocks(int64_t n);

}  // namespace mxp
