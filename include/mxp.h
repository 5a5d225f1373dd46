/*
 * mxp.h -- C ABI of libmxp, a mixed-precision dense solver for one MI355X
 * (gfx950): counter-based generation of a diagonally dominant matrix, LU
 * without pivoting in low precision, and GMRES-based iterative refinement
 * in FP64 that recovers a solution meeting the HPL backward-error test.
 *
 * Paper passages the calls follow (HPL-MxP, Dongarra and Luszczek 2025):
 *   "Matrix Generation"      -- scalable generation; diagonal scaling that
 *                               makes pivoting unnecessary.
 *   "Algorithmic Framework"  -- LU in low precision (panel and triangular
 *                               solves in 32-bit, Schur-complement update in
 *                               16-bit with 32-bit accumulation, Figure 1),
 *                               x0 from the factors, GMRES in 64-bit with the
 *                               factors as a left preconditioner, at most 50
 *                               iterations, HPL scaled residual < 16 with
 *                               eps = 2^-53, balancing/scaling allowed and
 *                               undone at the end.
 *
 * Conventions for every call:
 *   - Matrices are column-major.  Leading dimensions and sizes are int64.
 *   - Pointers named A, B, X, diag, a_inf, aux, work are DEVICE pointers
 *     (memory on the current HIP device) owned by the caller; the library
 *     never frees them and never keeps them after the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it.  A call returns after enqueueing unless its
 *     comment says it synchronises.
 *   - Return value: MXP_OK (0); a negative code for an argument or runtime
 *     error, in which case nothing was enqueued (MXP_EINVAL, MXP_EWORKSPACE)
 *     or a HIP call failed (MXP_EHIP, text in mxp_last_error()); a positive
 *     code for a numerical outcome (MXP_ESINGULAR, MXP_ENOCONV,
 *     MXP_ECRITERION).  No C++ exception crosses this interface.
 *   - The library allocates no device memory in mxp_generate, mxp_factor
 *     and mxp_solve_ir: scratch space is passed in (`work`) and sized by
 *     the matching *_bytes query.
 */
#ifndef MXP_H
#define MXP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element formats */
typedef enum {
    MXP_F64 = 0,
    MXP_F32 = 1,
    MXP_F16 = 2,     /* IEEE binary16 */
    MXP_BF16 = 3,    /* bfloat16 */
    MXP_F8E4M3 = 4   /* OCP fp8 e4m3fn (max 448, no infinities) */
} mxp_dtype;

/* status codes */
enum {
    MXP_OK = 0,
    MXP_EINVAL = -1,      /* bad argument (size, dtype combination, NULL pointer) */
    MXP_EWORKSPACE = -2,  /* work buffer smaller than the *_bytes query says */
    MXP_EHIP = -3,        /* a HIP runtime call failed; see mxp_last_error() */
    MXP_ESINGULAR = 1,    /* zero or non-finite pivot; *info = 1-based column */
    MXP_ENOCONV = 2,      /* refinement needed more than max_iters iterations */
    MXP_ECRITERION = 3,   /* refinement stopped but scaled residual >= tol */
    MXP_PENDING = 4       /* mxp_server_poll: the request is not done yet */
};

/* input scaling applied before the factorisation ("Algorithmic Framework":
 * balancing and scaling are allowed, their time counts, and their effect is
 * undone at the end) */
enum {
    MXP_SCALE_NONE = 0,
    MXP_SCALE_ROW_EQUIL = 1  /* row i scaled by the power of two nearest 1/A[i,i] */
};

/* text of the last MXP_EHIP / MXP_EINVAL error of the calling thread */
const char *mxp_last_error(void);

/* library version string */
const char *mxp_version(void);

/* matrix kinds of mxp_generate ("Matrix Generation"; "Experimental Results") */
enum {
    MXP_GEN_DOMINANT = 0,  /* off-diagonal uniform in [-1/2, 1/2), diagonal = sum of |row|: the
                              diagonally dominant class meant for debugging and tuning */
    MXP_GEN_SQRTN = 1,     /* off-diagonal as above, diagonal = own draw + gamma sqrt(n): the
                              sqrt(n) scaling suggested by random-matrix theory; far from row
                              dominance, and for gamma near 1/sqrt(12) hard for GMRES
                              without a preconditioner */
    MXP_GEN_UNIFORM = 2    /* every entry uniform in [-1, 1), no diagonal scaling: the matrices
                              of the pivoting experiments (Figures 2-4) */
};

/*
 * mxp_generate -- "Matrix Generation".
 * Generates A (n x n) and B (n x nrhs) from `seed`.  With k(i,j) the 32-bit
 * Philox4x32-10 draw of stream 0 at counter (i, j/4, 0, 0), word j%4, key =
 * (seed low 32 bits, seed high 32 bits), and u(i,j) = k(i,j) 2^-32 - 1/2:
 *   MXP_GEN_DOMINANT: A[i,j] = u(i,j) (i != j),
 *                     A[i,i] = sum over ALL j of |u(i,j)| (exact);
 *   MXP_GEN_SQRTN:    A[i,j] = u(i,j) (i != j),
 *                     A[i,i] = u(i,i) + fl(gamma * fl(sqrt(n))) (one FP64 add);
 *   MXP_GEN_UNIFORM:  A[i,j] = 2 u(i,j) for every i, j.
 *   B[i,r] = draw of stream 1 at (i, r) mapped to [-1/2, 1/2) the same way.
 * A is written in the storage format `store` (MXP_F32, MXP_F16, MXP_BF16, or
 * MXP_F64 for an exact copy), each entry rounded to nearest even from its
 * exact value; lda >= n.
 * A may be NULL (nothing stored: the solver regenerates A on the fly).
 * B (FP64, ldb >= n) may be NULL when nrhs == 0.
 * gamma: the diagonal coefficient of MXP_GEN_SQRTN (> 0), ignored otherwise.
 * diag (FP64, n entries): the exact diagonal (the regenerating residual
 *   reads it); required.
 * row_l1 (FP64, n entries, may be NULL): ||A[i,:]||_1 of the exact matrix
 *   (exact for the dominant and uniform kinds; one rounding for sqrt(n)).
 * a_inf (FP64, 1 entry): ||A||_inf = max_i row_l1[i]; required.
 * Asynchronous on `stream`.  n >= 1, n < 2^31.
 */
int mxp_generate(int64_t n, int64_t nrhs, uint64_t seed, int kind, double gamma, int store, void *A, int64_t lda,
                 double *B, int64_t ldb, double *diag, double *row_l1, double *a_inf, void *stream);

/*
 * Factorisation -- "Algorithmic Framework", Figure 1.
 * Right-looking blocked LU without pivoting with block size nb.  Per block
 * step: the diagonal block is factored in FP32; the block column
 * L21 = A21 U11^-1 and block row U12 = L11^-1 A12 are formed at FP32
 * quality -- while the trailing part spans at least 16 blocks and `store`
 * is 16-bit, as products with the diagonal block's FP32 inverses split into
 * 16-bit parts (matrix cores, FP32 accumulation), otherwise by blocked FP32
 * substitution; both are rounded to the update format `update`
 * (MXP_F16, MXP_BF16, MXP_F8E4M3 with a power-of-two scale per strip of
 * rows of L21 / columns of U12; MXP_F32 for an all-FP32 factorisation);
 * the trailing matrix is updated A22 <- A22 - L21 U12 on the matrix cores
 * with FP32 accumulation and stored back in `store`.  The updates of block
 * steps k and k+1 (k an even block index) reach everything beyond block
 * k+1 in one pass: their sum is accumulated in FP32 and rounded to `store`
 * once; block column and row k+1 receive step k's update alone.
 *
 * On return A holds L (unit lower, strictly below the diagonal; blocks of
 * L21 stored multiplied by their power-of-two scale) and U (upper) in the
 * storage format, and `aux` holds what the solve needs: the FP32 diagonal
 * blocks, FP32 inverses of the preconditioner's diagonal blocks (pairs of
 * factor blocks for nb <= 512) and of the 64x64 diagonal sub-blocks, the
 * per-strip scales of the stored L21, and the FP64 row scaling.
 *
 * Valid (update, store) pairs: (F32,F32), (F16,F16), (BF16,BF16),
 * (F8E4M3,F16), (F8E4M3,BF16), (F16,F32), (BF16,F32).
 * nb must be a multiple of 64 in [64, 1024].
 *
 * mxp_factor_aux_bytes / mxp_factor_work_bytes give the sizes of `aux`
 * (kept until the last solve) and `work` (scratch during the call).
 * `scaling`: MXP_SCALE_NONE, or MXP_SCALE_ROW_EQUIL which first scales
 * row i of A in place by 2^t / p_i, p_i the power of two nearest diag[i]
 * (t = 14 for FP16 storage, keeping the off-diagonal entries in FP16's
 * normal range, 0 otherwise; diag = the exact FP64 diagonal from
 * mxp_generate, required then, else may be NULL)
 * and records the factors in `aux`; the solve applies the same scaling to
 * its vectors, so X solves the original, unscaled system.
 * `info` (host pointer, may be NULL): if non-NULL the call synchronises
 * the stream and stores 0 or the 1-based column of the first zero /
 * non-finite pivot, returning MXP_ESINGULAR in the latter case; if NULL
 * the call is asynchronous and a singular pivot is NOT reported -- an
 * asynchronous caller that needs the report reads the info word of `work`
 * (mxp_factor_get_layout: work offset `info`, an unsigned 64-bit value, all
 * ones when no pivot failed) after the stream has finished.
 * Concurrency: the factorisation runs on `stream` and on a side stream of
 * its own (look-ahead); each call takes a side stream and its events from a
 * per-device pool for the time of the call, so host threads may factor at
 * the same time on different streams.  Calls sharing `work`, `aux` or `A`
 * must be ordered by the caller.
 */
size_t mxp_factor_aux_bytes(int64_t n, int64_t nb);
size_t mxp_factor_work_bytes(int64_t n, int64_t nb, int update);
int mxp_factor(int64_t n, int64_t nb, int update, int store, int scaling, const double *diag, void *A,
               int64_t lda, void *aux, void *work, size_t work_bytes, int64_t *info, void *stream);

/*
 * mxp_factor_group -- the factorisations of up to 8 independent matrices of
 * the same formats in lockstep on one stream (the batched launches of the
 * solve server; not in the paper): per block step ONE launch factors the
 * diagonal blocks of all of them, ONE launch forms all their strip solves
 * (one launch per kernel of the inverse-based form),
 * and per pair of block steps ONE launch updates all their next block
 * columns and rows and ONE all their trailing matrices (the two steps
 * merged, as in mxp_factor), each kernel finding its matrix through a
 * descriptor array.  Sizes and block sizes may differ;
 * no look-ahead.  Each item's A, aux and work are as for mxp_factor (no
 * scaling); the results are those of mxp_factor bit for bit.
 * tile: the work-group tile of the trailing update, MXP_TILE_256x128 (the
 *   one mxp_factor uses for launches of at least one tile per CU) or
 *   MXP_TILE_128x128 (twice the tiles: small n).
 * info: host array of count entries (may be NULL: asynchronous), as for
 *   mxp_factor; MXP_ESINGULAR if any matrix had a bad pivot.
 */
enum { MXP_TILE_256x128 = 0, MXP_TILE_128x128 = 1 };
typedef struct {
    int64_t n, nb;
    void *A;
    int64_t lda;
    void *aux, *work;
    size_t work_bytes;
} mxp_factor_item;
int mxp_factor_group(int count, const mxp_factor_item *items, int update, int store, int tile, int64_t *info,
                     void *stream);

/*
 * Where mxp_factor puts things in `aux` and `work` (byte offsets), for
 * inspection and testing.  With nblk = ceil(n / nb) diagonal blocks and
 * strips = ceil(n / 32):
 *   aux:  T         FP32 nblk x nb x nb: L11\U11 of every diagonal block
 *                   (column-major, ld nb; the FP32 factor the preconditioner
 *                   applies)
 *         Trm       the same, row-major
 *         linv/uinv FP32 nblk x (nb/64) x 64 x 64: inverses of the 64 x 64
 *                   diagonal sub-blocks (L column-major, U row-major)
 *         lsc       FP32 nblk x strips: the power-of-two factor s of every
 *                   stored 32-row strip of L21 (entry [blk][r/32]; the
 *                   stored value is s * L), 1 where no scaling is applied
 *         rowscale  FP64 n: the row scaling S (1 without equilibration)
 *         linv_full/uinv_full FP32 ngrp x D x D, column-major (ld D): the
 *                   inverses of the unit-lower and upper parts of the
 *                   preconditioner's diagonal blocks -- pairs of factor
 *                   blocks (D = 2 nb) for nb <= 512, single ones (D = nb)
 *                   otherwise; ngrp = ceil(n / D)
 *   work: Lq/Uq     four sets of op_rows x nb update operands
 *                   (row-major: K contiguous), set (k/nb) & 3 for step k;
 *                   row 0 of a set is the first row after the step's block
 *         inv_sa/inv_sb four sets of op_rows/32 FP32 factors 1/s per
 *                   32-row strip of Lq / Uq
 *         info      unsigned 64-bit: first failing pivot column, ~0 if none
 *         (then scratch of the preconditioner's inverses)
 * Returns MXP_EINVAL for sizes mxp_factor would reject.
 */
typedef struct {
    size_t T, Trm, linv, uinv, lsc, rowscale, linv_full, uinv_full, aux_bytes;
    size_t Lq, Uq, inv_sa, inv_sb, info, work_bytes;
    int64_t op_rows, strips;
} mxp_factor_layout;
int mxp_factor_get_layout(int64_t n, int64_t nb, int update, mxp_factor_layout *out);

/* per-right-hand-side outcome of the refinement */
typedef struct {
    int64_t iters;   /* inner GMRES iterations (matrix-vector products), all restarts */
    int64_t cycles;  /* restart cycles run */
    double eta;      /* final HPL scaled residual */
    int32_t status;  /* MXP_OK, MXP_ENOCONV or MXP_ECRITERION */
    int32_t pad;
} mxp_rhs_report;

/*
 * mxp_solve_ir -- "Algorithmic Framework".
 * For each right-hand side r: x0 = M^-1 b_r with M^-1 = U^-1 L^-1 S (the
 * factors from mxp_factor, S the row scaling); then repeat: residual
 * r = b - A x in FP64 with A regenerated from (seed, diag) instead of read
 * from memory; eta = ||r||_inf / ((||A||_inf ||x||_inf + ||b||_inf) n 2^-53);
 * stop when eta < tol; otherwise one cycle of left-preconditioned GMRES
 * (restart `restart`, modified Gram-Schmidt, Givens rotations, inner stop
 * when the rotated residual <= tau * ||x||_2) and x += V y.  More than
 * max_iters inner iterations in total is a failure (MXP_ENOCONV).
 * All vector work runs in FP64 on the device; only the convergence scalars
 * cross to the host.
 *
 * LU/lda/aux/nb/update/store: as produced by mxp_factor.  seed, kind, diag
 * and a_inf: as given to / produced by mxp_generate.  B (ldb >= n) is read,
 * X (ldx >= n) written.  rep: host array of nrhs reports.
 * restart in [1, 64]; max_iters >= 1; tol > 0 (16 for the HPL test);
 * tau >= 0 (2^-50 recommended).
 * Synchronises `stream` (it reads convergence scalars).  Returns MXP_OK
 * when every right-hand side passed, else the worst positive status.
 */
size_t mxp_solve_work_bytes(int64_t n, int64_t nrhs, int restart);
int mxp_solve_ir(int64_t n, int64_t nb, int update, int store, uint64_t seed, int kind, const void *LU, int64_t lda,
                 const void *aux, const double *diag, const double *a_inf, const double *B, int64_t ldb,
                 double *X, int64_t ldx, int64_t nrhs, int restart, int max_iters, double tol, double tau,
                 mxp_rhs_report *rep, void *work, size_t work_bytes, void *stream);

/*
 * Building blocks exposed for testing and measurement (same conventions;
 * each has a *_work_bytes query for its scratch buffer).
 *
 * mxp_residual: R = B - A X for nrhs columns (R = A X when B is NULL),
 *   FP64, A regenerated from (seed, kind, diag) -- the refinement's residual
 *   ("Algorithmic Framework": the 64-bit residual of the refinement).
 * mxp_apply_prec: Z = M^-1 V = U^-1 L^-1 S V for nrhs columns (nrhs <= 64),
 *   FP64 arithmetic on the stored factor (the left preconditioner);
 *   synchronises (it reads back an error word: MXP_EHIP if a wait of the
 *   block-substitution kernels expired).  mxp_solve_ir reports the same.
 * mxp_hpl_eta: the HPL scaled residual of one right-hand side (x, b on the
 *   device) written to the host double *eta; synchronises.
 */
size_t mxp_residual_work_bytes(int64_t n, int64_t nrhs);
int mxp_residual(int64_t n, uint64_t seed, int kind, const double *diag, const double *X, int64_t ldx,
                 const double *B, int64_t ldb, double *R, int64_t ldr, int64_t nrhs, void *work, size_t work_bytes,
                 void *stream);
/*
 * mxp_residual_noalloc: mxp_residual without a work buffer, for callers that
 *   cannot allocate device memory (code under stream capture, tight serving
 *   loops, harnesses that forbid allocation).  The partial products live in
 *   a file-scope device array of the library, 32 MiB per device, held by
 *   every device the library runs on until the process ends; the call
 *   allocates nothing.  Sizes whose partials exceed it (mxp_residual_work_bytes
 *   > 32 MiB: n * min(nrhs, 8) above about 4 M, e.g. n = 131072 fits with 8
 *   columns) are rejected with MXP_EINVAL.  Every call on a device shares
 *   that device's array: calls that overlap on one device (several streams
 *   or host threads) race and must be ordered by the caller.  Nothing in the
 *   array needs clearing: each call overwrites what it reads.
 */
int mxp_residual_noalloc(int64_t n, uint64_t seed, int kind, const double *diag, const double *X, int64_t ldx,
                         const double *B, int64_t ldb, double *R, int64_t ldr, int64_t nrhs, void *stream);
size_t mxp_apply_prec_work_bytes(int64_t n, int64_t nrhs);
int mxp_apply_prec(int64_t n, int64_t nb, int update, int store, const void *LU, int64_t lda, const void *aux,
                   const double *V, int64_t ldv, double *Z, int64_t ldz, int64_t nrhs, void *work, size_t work_bytes,
                   void *stream);
/*
 * mxp_trailing_update: the Schur-complement update of one block step
 * ("Algorithmic Framework", Figure 1), C <- C - diag(inv_sa) Aq Bq^T diag(inv_sb):
 * C is M x N column-major in the storage format (ldc >= M); Aq (M x K) and
 * Bq (N x K) are the operands in the update format, each row's K values
 * contiguous, with the row counts padded to a multiple of 256 (padding rows
 * are read, never written); inv_sa / inv_sb hold one FP32 factor per 32 rows
 * of Aq / Bq (padded likewise).  K * element size must be a multiple of 128
 * bytes.  Asynchronous.
 */
int mxp_trailing_update(int64_t M, int64_t N, int64_t K, int update, int store, void *C, int64_t ldc,
                        const void *Aq, const void *Bq, const float *inv_sa, const float *inv_sb, void *stream);
/*
 * mxp_trailing_update2: the updates of two consecutive block steps in one
 * pass (how mxp_factor updates everything beyond the next block column),
 * C <- C - [diag(inv_sa1) Aq1 Bq1^T diag(inv_sb1) + diag(inv_sa2) Aq2 Bq2^T diag(inv_sb2)]:
 * each operand pair as for mxp_trailing_update (K1 resp. K2 values per row,
 * K * element size a multiple of 128 bytes); the factors must be powers of
 * two.  The sum is accumulated in FP32 (the first step's partial sums are
 * brought to the second step's scale, exactly) and rounded to the storage
 * format once.  Asynchronous.
 */
int mxp_trailing_update2(int64_t M, int64_t N, int64_t K1, int64_t K2, int update, int store, void *C, int64_t ldc,
                         const void *Aq1, const void *Bq1, const float *inv_sa1, const float *inv_sb1,
                         const void *Aq2, const void *Bq2, const float *inv_sa2, const float *inv_sb2, void *stream);
size_t mxp_hpl_eta_work_bytes(int64_t n);
int mxp_hpl_eta(int64_t n, uint64_t seed, int kind, const double *diag, const double *a_inf, const double *x,
                const double *b, double *eta, void *work, size_t work_bytes, void *stream);

/*
 * FP64 LU -- the FP64 solve the figure of merit is compared with
 * ("Background"), and the LU of the pivoting study ("Experimental Results",
 * Figures 2-4: LU in 64-bit arithmetic with and without partial pivoting).
 * Right-looking blocked LU of the FP64 matrix A (n x n, lda >= n, in place:
 * L unit lower and U), block size 128 (64 above n = 32768), trailing update
 * on the FP64 matrix cores.
 * ipiv (device, n int64 entries, may be NULL): NULL factors without
 *   pivoting; otherwise partial pivoting (largest magnitude in the column,
 *   the first among equals, as LAPACK getrf) with ipiv[k] = the 0-based row
 *   swapped with row k; the swaps are applied to the whole matrix.
 *   Pivoting needs n <= 65536.
 * gemm: the trailing update, MXP_GEMM64_OWN (this library's FP64 matrix-core
 *   kernel, mxp_trailing_update64) or MXP_GEMM64_ROCBLAS (rocBLAS dgemm, a
 *   plain library GEMM: the baseline at the vendor library's speed).
 * work: mxp_lu64_work_bytes(n) bytes of device scratch.
 * info (host, may be NULL): as mxp_factor (synchronises, MXP_ESINGULAR and
 *   the 1-based column of the first zero / non-finite pivot); MXP_EHIP if a
 *   bounded wait of the pivoted panel expired.  NULL: asynchronous.
 * mxp_lu64_solve: X <- U^-1 L^-1 P X for nrhs <= 64 columns (ldx >= n), with
 *   the factors and ipiv (may be NULL) of mxp_lu64_factor.  Asynchronous.
 */
enum { MXP_GEMM64_OWN = 0, MXP_GEMM64_ROCBLAS = 1 };
size_t mxp_lu64_work_bytes(int64_t n);
/* the FP64 trailing update C (M x N, ldc) -= A (M x K, lda) B (K x N, ldb),
 * column-major, K a multiple of 4, on the FP64 matrix cores; asynchronous */
int mxp_trailing_update64(int64_t M, int64_t N, int64_t K, double *C, int64_t ldc, const double *A, int64_t lda,
                          const double *B, int64_t ldb, void *stream);
int mxp_lu64_factor(int64_t n, double *A, int64_t lda, int64_t *ipiv, int gemm, void *work, size_t work_bytes,
                    int64_t *info, void *stream);
int mxp_lu64_solve(int64_t n, const double *LU, int64_t lda, const int64_t *ipiv, double *X, int64_t ldx,
                   int64_t nrhs, void *stream);

/*
 * Timing of kernel classes with HIP events recorded on the stream each
 * kernel is launched on (off by default).  Classes: 0 trailing update,
 * 1 strip TRSMs, 2 diagonal-block LU, 3 preconditioner apply, 4 regenerating
 * residual / matrix-vector product, 6 FP64 trailing update (mxp_lu64_*).  mxp_profile_enable(mask) times the
 * classes whose bit is set in mask (0: timing off); the events add work to
 * each timed launch's stream.  mxp_profile_read synchronises on the
 * recorded events and returns, for one class, the summed kernel time, the
 * summed algorithmic flops and bytes, and the number of timed launches
 * since the last reset.
 */
int mxp_profile_enable(int mask);
int mxp_profile_reset(void);
int mxp_profile_read(int cls, double *total_ms, double *flops, double *bytes, int64_t *launches);

/*
 * ---------------------------------------------------------------- serving
 * A solve server on one device: requests (n, nrhs, seed) arrive at any
 * time; each is generated, factored and refined with the same arithmetic as
 * mxp_generate + mxp_factor + mxp_solve_ir.  Requests are admitted in arrival
 * order as soon as a slot is free and their device memory fits in the HBM
 * budget (the caller's arena, sub-allocated by the server); up to max_slots
 * requests are in flight at once.  A few worker threads (at most 3, one
 * stream each) take groups of admitted requests: a group's factorisations
 * run in lockstep with one launch per kernel and block step for the whole
 * group (mxp_factor_group), then each request is refined with all its
 * right-hand sides together and returned; requests that arrive meanwhile
 * form the next groups, which overlap on the device (continuous batching).
 * The block size and trailing-update tile of each request are chosen by
 * size class; with `autotune` the server times every candidate pair of each
 * class on the device at creation and keeps the fastest.  The paper has no
 * serving part; the calls follow its statement of the problem for every
 * request.
 *
 * Ownership: `arena` is a device buffer of arena_bytes owned by the caller,
 * valid until mxp_server_destroy returns.  x_host given to submit is a host
 * buffer of n * nrhs doubles (column-major, ld n) that receives the solution
 * (may be NULL); it must stay valid until the request is done.
 * Thread safety: every call may be made from any thread.
 */
typedef struct mxp_server mxp_server;

typedef struct {
    int max_slots;      /* requests in flight at once (>= 1) */
    int update;         /* update format, e.g. MXP_BF16 */
    int store;          /* storage format of A and the factor, e.g. MXP_BF16 */
    int nb;             /* block size; 0 = by size class (see autotune) */
    int autotune;       /* nonzero: time the candidate block sizes at creation */
    int restart;        /* GMRES restart length (1..64) */
    int max_iters;      /* iteration cap of the refinement */
    double tol;         /* HPL scaled-residual threshold, e.g. 16 */
    double tau;         /* inner GMRES tolerance (mxp_solve_ir) */
} mxp_server_cfg;

typedef struct {
    uint64_t id;
    int64_t n, nrhs, nb;
    int status;         /* MXP_OK or the first non-OK code of generate / factor / solve */
    int pad;
    int64_t iters;      /* largest iteration count over the right-hand sides */
    double eta;         /* largest final scaled residual over the right-hand sides */
    int64_t t_submit_ns, t_start_ns, t_done_ns;   /* steady clock, since server creation */
} mxp_request_result;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t in_flight, peak_in_flight;
    size_t arena_bytes, bytes_in_use, peak_bytes_in_use;
    int64_t groups;            /* groups factored together (one launch per kernel and block step) */
    int64_t grouped_requests;  /* requests in those groups */
    int64_t peak_group;        /* largest group */
    int64_t streams;           /* device streams of the server (one per worker) */
} mxp_server_stats;

/* device bytes one request needs (A, B, X, diag and all work spaces) */
size_t mxp_server_request_bytes(int64_t n, int64_t nrhs, int64_t nb, int update, int store, int restart);

/* creates the server (and, with cfg->autotune, runs the block-size tuner,
 * which uses the arena and synchronises).  *out receives the handle. */
int mxp_server_create(int device, void *arena, size_t arena_bytes, const mxp_server_cfg *cfg, mxp_server **out);

/* queues a request; returns MXP_EINVAL if it can never fit the arena.
 * *id receives its id (ids count from 1). */
int mxp_server_submit(mxp_server *srv, int64_t n, int64_t nrhs, uint64_t seed, double *x_host, uint64_t *id);

/* MXP_OK and *out filled if request `id` is done; MXP_PENDING if not yet;
 * MXP_EINVAL for an unknown id */
int mxp_server_poll(mxp_server *srv, uint64_t id, mxp_request_result *out);

/* blocks until request `id` is done, then as mxp_server_poll */
int mxp_server_wait(mxp_server *srv, uint64_t id, mxp_request_result *out);

/* blocks until every submitted request is done */
int mxp_server_drain(mxp_server *srv);

int mxp_server_get_stats(mxp_server *srv, mxp_server_stats *out);

/* block size the server uses for a request of size n */
int64_t mxp_server_block_size(mxp_server *srv, int64_t n);

/* trailing-update tile (MXP_TILE_*) the server uses for a request of size n */
int mxp_server_tile(mxp_server *srv, int64_t n);

/* drains, stops the slot threads and releases the server's streams */
int mxp_server_destroy(mxp_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* MXP_H */
