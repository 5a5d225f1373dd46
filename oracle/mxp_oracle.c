/*
 * mxp_oracle.c -- plain, slow, CPU reference for the HPL-MxP solve path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * What it computes (paper: "Algorithmic Framework" and "Matrix Generation"):
 *   - a counter-based random matrix A whose off-diagonal entries are uniform
 *     in (-1/2, 1/2) and whose diagonal is the sum of |row|, so that A is
 *     row diagonally dominant and admits an LU factorisation without
 *     pivoting ("Matrix Generation": scalable generation, and the diagonal
 *     scaling that makes pivoting unnecessary);
 *   - unpivoted LU in FP64 (textbook right-looking elimination, no blocking);
 *   - forward / backward substitution;
 *   - restarted GMRES with the LU factors as a LEFT preconditioner, used as
 *     a non-stationary iterative refinement in FP64 ("Algorithmic Framework");
 *   - the HPL scaled residual ||Ax-b||_inf / ((||A||_inf ||x||_inf + ||b||_inf) n eps)
 *     with eps = 2^-53, valid when < 16 ("Algorithmic Framework", the
 *     backward-error formula);
 *   - a Jacobi iteration with A regenerated row by row, which reaches the
 *     same x = A^-1 b with O(n) memory for sizes the dense LU cannot hold
 *     (strict row diagonal dominance makes Jacobi converge);
 *   - round-to-nearest-even conversions of FP64 values to the storage and
 *     operand formats (fp32, fp16, bf16, fp8 e4m3fn), written from the
 *     format definitions.
 *
 * Readings of points the paper leaves open (the random generator, the
 * meaning of "iterations" in the 50-iteration cap, the inner tolerance) are
 * those listed in the design notes of the repository.
 *
 * Random numbers: Philox4x32-10, from Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011, section 3.3: the Philox S-box with    */
/* two 32x32->64 multiplications per round and a Weyl-sequence key bump).   */
/* ------------------------------------------------------------------------ */

#define PHILOX_MUL0 0xD2511F53u
#define PHILOX_MUL1 0xCD9E8D57u
#define PHILOX_WEYL0 0x9E3779B9u
#define PHILOX_WEYL1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* the key is bumped between rounds */
            k0 += PHILOX_WEYL0;
            k1 += PHILOX_WEYL1;
        }
        uint64_t p0 = (uint64_t)PHILOX_MUL0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_MUL1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * The raw 32-bit draw for stream s at (row i, column j).
 * Counter = (i, j/4, s, 0), key = (low 32 bits of seed, high 32 bits),
 * and the draw is output word j mod 4.  Stream 0 is the matrix, stream 1
 * the right-hand sides (j = right-hand-side index).
 */
uint32_t orc_draw(uint64_t seed, uint32_t stream, int64_t i, int64_t j)
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(j >> 2), stream, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[j & 3];
}

/* value of a draw: k * 2^-32 - 1/2, exactly representable in FP64 */
static double draw_value(uint32_t k)
{
    return ldexp((double)k, -32) - 0.5;
}

/*
 * Matrix kinds ("Matrix Generation"; "Experimental Results"):
 *   0 dominant: off-diagonal u(i,j) = draw value in [-1/2, 1/2); diagonal =
 *     the sum over the whole row (own draw included) of |u(i,j)|;
 *   1 sqrt(n):  off-diagonal u(i,j); diagonal = u(i,i) + gamma * sqrt(n)
 *     (each operation rounded once in FP64);
 *   2 uniform:  every entry 2 u(i,j), in [-1, 1), no diagonal change.
 */
typedef struct {
    int64_t n;
    uint64_t seed;
    int kind;
    double gamma;
} orc_gen;

/* the draw value u(i,j) of the matrix stream */
double orc_entry_draw(uint64_t seed, int64_t i, int64_t j)
{
    return draw_value(orc_draw(seed, 0u, i, j));
}

/* right-hand side entry b[i,r] */
double orc_rhs(uint64_t seed, int64_t i, int64_t r)
{
    return draw_value(orc_draw(seed, 1u, i, r));
}

/* off-diagonal entry A[i,j] (i != j) of a kind */
static double gen_offdiag(const orc_gen *g, int64_t i, int64_t j)
{
    double u = orc_entry_draw(g->seed, i, j);
    return g->kind == 2 ? 2.0 * u : u;
}

/* diagonal entry A[i,i] of a kind */
static double gen_diag(const orc_gen *g, int64_t i)
{
    if (g->kind == 1) {
        double shift = g->gamma * sqrt((double)g->n);
        return orc_entry_draw(g->seed, i, i) + shift;
    }
    if (g->kind == 2)
        return 2.0 * orc_entry_draw(g->seed, i, i);
    double s = 0.0;
    for (int64_t j = 0; j < g->n; ++j)
        s += fabs(orc_entry_draw(g->seed, i, j));
    return s;
}

double orc_diag(int64_t n, uint64_t seed, int kind, double gamma, int64_t i)
{
    orc_gen g = {n, seed, kind, gamma};
    return gen_diag(&g, i);
}

/* A[i,j] of the generated matrix, FP64 */
double orc_entry(int64_t n, uint64_t seed, int kind, double gamma, int64_t i, int64_t j)
{
    orc_gen g = {n, seed, kind, gamma};
    return (i == j) ? gen_diag(&g, i) : gen_offdiag(&g, i, j);
}

/* dense generation: A column-major (lda >= n), diag[n] and row_l1[n] (may be NULL) */
void orc_generate(int64_t n, uint64_t seed, int kind, double gamma, double *A, int64_t lda, double *diag,
                  double *row_l1)
{
    orc_gen g = {n, seed, kind, gamma};
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            A[i + j * lda] = (i == j) ? 0.0 : gen_offdiag(&g, i, j);
    for (int64_t i = 0; i < n; ++i) {
        double d = gen_diag(&g, i);
        A[i + i * lda] = d;
        if (diag) diag[i] = d;
        if (row_l1) {
            double off = 0.0;
            for (int64_t j = 0; j < n; ++j)
                if (j != i) off += fabs(A[i + j * lda]);
            row_l1[i] = off + fabs(d);
        }
    }
}

void orc_generate_rhs(int64_t n, int64_t nrhs, uint64_t seed, double *B, int64_t ldb)
{
    for (int64_t r = 0; r < nrhs; ++r)
        for (int64_t i = 0; i < n; ++i)
            B[i + r * ldb] = orc_rhs(seed, i, r);
}

/* ||A||_inf of the generated matrix, regenerating rows (O(n) memory) */
double orc_anorm_inf_regen(int64_t n, uint64_t seed, int kind, double gamma)
{
    orc_gen g = {n, seed, kind, gamma};
    double best = 0.0;
#pragma omp parallel for reduction(max : best) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double off = 0.0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i) off += fabs(gen_offdiag(&g, i, j));
        double row = off + fabs(gen_diag(&g, i));
        if (row > best) best = row;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Dense FP64 linear algebra (column-major)                                  */
/* ------------------------------------------------------------------------ */

double orc_norm_inf_mat(int64_t n, const double *A, int64_t lda)
{
    double best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            s += fabs(A[i + j * lda]);
        if (s > best) best = s;
    }
    return best;
}

static double norm_inf_vec(int64_t n, const double *x)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (fabs(x[i]) > m) m = fabs(x[i]);
    return m;
}

static double dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

static double norm2(int64_t n, const double *x)
{
    return sqrt(dot(n, x, x));
}

/* y = A x */
void orc_matvec(int64_t n, const double *A, int64_t lda, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double xj = x[j];
        for (int64_t i = 0; i < n; ++i) y[i] += A[i + j * lda] * xj;
    }
}

/*
 * Unpivoted LU, in place: on return the strict lower triangle holds L
 * (unit diagonal implied) and the upper triangle holds U.  Textbook
 * right-looking elimination: for each pivot k, scale the column below it,
 * then subtract the rank-one product from the trailing matrix.
 * Returns 0, or the 1-based index of the first zero / non-finite pivot.
 */
int64_t orc_lu_nopiv(int64_t n, double *A, int64_t lda)
{
    for (int64_t k = 0; k < n; ++k) {
        double piv = A[k + k * lda];
        if (piv == 0.0 || !isfinite(piv)) return k + 1;
        for (int64_t i = k + 1; i < n; ++i) A[i + k * lda] /= piv;
        for (int64_t j = k + 1; j < n; ++j) {
            double ukj = A[k + j * lda];
            if (ukj == 0.0) continue;
            for (int64_t i = k + 1; i < n; ++i)
                A[i + j * lda] -= A[i + k * lda] * ukj;
        }
    }
    return 0;
}

/*
 * LU with partial pivoting, in place ("Experimental Results": the standard
 * FP64 factorisation whose largest pivot Figure 2 reports): for each column
 * k the entry of largest magnitude on or below the diagonal (the first one
 * among equals) becomes the pivot, rows k and p are swapped across the whole
 * matrix, then the column is scaled and the trailing matrix updated.
 * ipiv[k] = p (0-based row swapped with k).  Returns 0, or the 1-based index
 * of the first zero pivot (the elimination goes on past it without scaling).
 */
int64_t orc_lu_pp(int64_t n, double *A, int64_t lda, int64_t *ipiv)
{
    int64_t info = 0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = k;
        double best = fabs(A[k + k * lda]);
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(A[i + k * lda]) > best) { best = fabs(A[i + k * lda]); p = i; }
        ipiv[k] = p;
        if (p != k)
            for (int64_t j = 0; j < n; ++j) {
                double t = A[k + j * lda];
                A[k + j * lda] = A[p + j * lda];
                A[p + j * lda] = t;
            }
        double piv = A[k + k * lda];
        if (piv == 0.0) {
            if (!info) info = k + 1;
            continue;
        }
        for (int64_t i = k + 1; i < n; ++i) A[i + k * lda] /= piv;
        for (int64_t j = k + 1; j < n; ++j) {
            double ukj = A[k + j * lda];
            if (ukj == 0.0) continue;
            for (int64_t i = k + 1; i < n; ++i)
                A[i + j * lda] -= A[i + k * lda] * ukj;
        }
    }
    return info;
}

/* x <- P x with the row swaps ipiv of orc_lu_pp, in order */
void orc_apply_pivots(int64_t n, const int64_t *ipiv, double *x)
{
    for (int64_t k = 0; k < n; ++k) {
        double t = x[k];
        x[k] = x[ipiv[k]];
        x[ipiv[k]] = t;
    }
}

/* x <- L^-1 x (L unit lower in LU), then x <- U^-1 x */
void orc_lu_solve(int64_t n, const double *LU, int64_t lda, double *x)
{
    for (int64_t j = 0; j < n; ++j) {          /* forward, column oriented */
        double xj = x[j];
        for (int64_t i = j + 1; i < n; ++i) x[i] -= LU[i + j * lda] * xj;
    }
    for (int64_t j = n - 1; j >= 0; --j) {     /* backward, column oriented */
        x[j] /= LU[j + j * lda];
        double xj = x[j];
        for (int64_t i = 0; i < j; ++i) x[i] -= LU[i + j * lda] * xj;
    }
}

/* HPL scaled residual (backward error), eps = 2^-53 */
double orc_hpl_eta(int64_t n, const double *A, int64_t lda, const double *x, const double *b)
{
    double *r = (double *)malloc((size_t)n * sizeof(double));
    orc_matvec(n, A, lda, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double eps = ldexp(1.0, -53);
    double eta = norm_inf_vec(n, r) /
                 ((orc_norm_inf_mat(n, A, lda) * norm_inf_vec(n, x) + norm_inf_vec(n, b)) * (double)n * eps);
    free(r);
    return eta;
}

/* r_i = b_i - (A x)_i for one row, A regenerated entry by entry (for the
 * dominant kind the diagonal's sum of |u| is taken in the same pass) */
static double residual_row(const orc_gen *g, int64_t i, const double *x, const double *b)
{
    double ax = 0.0, d;
    if (g->kind == 0) {
        double dsum = 0.0;
        for (int64_t j = 0; j < g->n; ++j) {
            double a = orc_entry_draw(g->seed, i, j);
            dsum += fabs(a);
            if (j != i) ax += a * x[j];
        }
        d = dsum;
    } else {
        for (int64_t j = 0; j < g->n; ++j)
            if (j != i) ax += gen_offdiag(g, i, j) * x[j];
        d = gen_diag(g, i);
    }
    return b[i] - (ax + d * x[i]);
}

/* r = b - A x with A regenerated entry by entry (rows in parallel) */
void orc_residual_regen(int64_t n, uint64_t seed, int kind, double gamma, const double *x, const double *b,
                        double *r)
{
    orc_gen g = {n, seed, kind, gamma};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        r[i] = residual_row(&g, i, x, b);
}

/* the same residual for the m sampled rows rows[0..m-1] only: out[k] = r[rows[k]] */
void orc_residual_rows(int64_t n, uint64_t seed, int kind, double gamma, const double *x, const double *b,
                       const int64_t *rows, int64_t m, double *out)
{
    orc_gen g = {n, seed, kind, gamma};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k)
        out[k] = residual_row(&g, rows[k], x, b);
}

/* HPL scaled residual with A regenerated (O(n) memory); a_inf < 0: computed here */
double orc_hpl_eta_regen(int64_t n, uint64_t seed, int kind, double gamma, const double *x, const double *b,
                         double a_inf)
{
    double *r = (double *)malloc((size_t)n * sizeof(double));
    orc_residual_regen(n, seed, kind, gamma, x, b, r);
    if (a_inf < 0) a_inf = orc_anorm_inf_regen(n, seed, kind, gamma);
    double eps = ldexp(1.0, -53);
    double eta = norm_inf_vec(n, r) / ((a_inf * norm_inf_vec(n, x) + norm_inf_vec(n, b)) * (double)n * eps);
    free(r);
    return eta;
}

/*
 * Jacobi iteration x <- D^-1 (b - (A - D) x), A regenerated row by row.
 * Converges for strictly row diagonally dominant A (the dominant kind).
 * Stops when the update is at most tol * ||x||_inf or after max_sweeps.
 * Returns the sweeps done.
 */
/* the diagonal A[i,i] of every row, d[n] */
void orc_diag_all(int64_t n, uint64_t seed, int kind, double gamma, double *d)
{
    orc_gen g = {n, seed, kind, gamma};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        d[i] = gen_diag(&g, i);
}

/* One Jacobi sweep from x, in place: x_i <- (b_i - sum_{j != i} A_ij x_j) / d_i
 * with the off-diagonal entries regenerated and d the diagonal
 * (orc_diag_all); returns max_i |x_new_i - x_old_i|. */
double orc_jacobi_sweep_regen(int64_t n, uint64_t seed, int kind, double gamma, const double *d, const double *b,
                              double *x)
{
    orc_gen g = {n, seed, kind, gamma};
    double *xn = (double *)malloc((size_t)n * sizeof(double));
    double dmax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : dmax)
    for (int64_t i = 0; i < n; ++i) {
        double off = 0.0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i) off += gen_offdiag(&g, i, j) * x[j];
        xn[i] = (b[i] - off) / d[i];
        double u = fabs(xn[i] - x[i]);
        if (u > dmax) dmax = u;
    }
    memcpy(x, xn, (size_t)n * sizeof(double));
    free(xn);
    return dmax;
}

int64_t orc_jacobi_regen(int64_t n, uint64_t seed, int kind, double gamma, const double *b, double *x,
                         int64_t max_sweeps, double tol)
{
    double *d = (double *)malloc((size_t)n * sizeof(double));
    int64_t sweeps = 0;
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    orc_diag_all(n, seed, kind, gamma, d);
    while (sweeps < max_sweeps) {
        const double dmax = orc_jacobi_sweep_regen(n, seed, kind, gamma, d, b, x);
        ++sweeps;
        if (dmax <= tol * norm_inf_vec(n, x)) break;
    }
    free(d);
    return sweeps;
}

/* ------------------------------------------------------------------------ */
/* GMRES-based iterative refinement with a left preconditioner              */
/* ------------------------------------------------------------------------ */

/*
 * The preconditioner is M^-1 v = U^-1 L^-1 v with L\U the packed factors in
 * PREC (which may be the FP64 factors or any other approximation of A), and
 * the operator is A itself (dense, FP64, the original matrix).
 */
typedef struct {
    int64_t n;
    const double *A; int64_t lda;
    const double *P; int64_t ldp;
} orc_system;

static void apply_prec(const orc_system *s, const double *v, double *z)
{
    memcpy(z, v, (size_t)s->n * sizeof(double));
    if (s->P) orc_lu_solve(s->n, s->P, s->ldp, z);
}

/*
 * One restart cycle of left-preconditioned GMRES from x, with modified
 * Gram-Schmidt and Givens rotations (Saad and Schultz 1986).  V is n x (m+1)
 * (column-major, ldv = n), H is (m+1) x m (column-major, ldh = m+1).
 * Iteration budget: *it counts matrix-vector products across cycles and
 * the cycle stops when *it reaches max_iters.  The cycle ends early when the
 * rotated residual |g_{k+1}| <= tau * ||x||_2.  Returns the Krylov
 * dimension used (0 if no step was taken) and updates x in place.
 * If keep_vh is nonzero V and H are left holding the Arnoldi basis and the
 * unrotated Hessenberg matrix (for tests), otherwise scratch.
 */
int64_t orc_gmres_cycle(int64_t n, const double *A, int64_t lda, const double *P, int64_t ldp,
                        const double *b, double *x, int64_t m, double tau, int64_t *it, int64_t max_iters,
                        double *V, double *H, double *Hraw, double *gout)
{
    orc_system s = {n, A, lda, P, ldp};
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    double *cs = (double *)calloc((size_t)m + 1, sizeof(double));
    double *sn = (double *)calloc((size_t)m + 1, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *y = (double *)calloc((size_t)m + 1, sizeof(double));
    int64_t ldh = m + 1;

    /* z = M^-1 (b - A x), beta = ||z||, v1 = z / beta, g = beta e1 */
    orc_matvec(n, A, lda, x, r);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    apply_prec(&s, r, w);
    double beta = norm2(n, w);
    int64_t k = 0;
    if (beta == 0.0) goto done;
    for (int64_t i = 0; i < n; ++i) V[i] = w[i] / beta;
    g[0] = beta;
    double xnorm = norm2(n, x);

    for (int64_t j = 0; j < m; ++j) {
        if (*it >= max_iters) break;
        *it += 1;
        /* w = M^-1 A v_j */
        orc_matvec(n, A, lda, V + j * n, r);
        apply_prec(&s, r, w);
        /* modified Gram-Schmidt */
        for (int64_t i = 0; i <= j; ++i) {
            double h = dot(n, V + i * n, w);
            H[i + j * ldh] = h;
            for (int64_t t = 0; t < n; ++t) w[t] -= h * V[t + i * n];
        }
        double hnext = norm2(n, w);
        H[j + 1 + j * ldh] = hnext;
        if (Hraw)
            for (int64_t i = 0; i <= j + 1; ++i) Hraw[i + j * ldh] = H[i + j * ldh];
        k = j + 1;
        if (hnext != 0.0)
            for (int64_t t = 0; t < n; ++t) V[t + (j + 1) * n] = w[t] / hnext;
        /* apply the previous rotations to the new column */
        for (int64_t i = 0; i < j; ++i) {
            double a = H[i + j * ldh], c = H[i + 1 + j * ldh];
            H[i + j * ldh] = cs[i] * a + sn[i] * c;
            H[i + 1 + j * ldh] = -sn[i] * a + cs[i] * c;
        }
        /* new rotation that zeroes H[j+1, j] */
        double a = H[j + j * ldh], c = H[j + 1 + j * ldh];
        double rho = hypot(a, c);
        cs[j] = a / rho;
        sn[j] = c / rho;
        H[j + j * ldh] = rho;
        H[j + 1 + j * ldh] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        if (hnext == 0.0) break;                 /* happy breakdown: exact */
        if (fabs(g[j + 1]) <= tau * xnorm) break;
    }
    /* back substitution y = R^-1 g, then x += V y */
    for (int64_t i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int64_t l = i + 1; l < k; ++l) t -= H[i + l * ldh] * y[l];
        y[i] = t / H[i + i * ldh];
    }
    for (int64_t i = 0; i < k; ++i)
        for (int64_t t = 0; t < n; ++t) x[t] += y[i] * V[t + i * n];
done:
    if (gout)
        for (int64_t i = 0; i <= m; ++i) gout[i] = g[i];
    free(r); free(w); free(cs); free(sn); free(g); free(y);
    return k;
}

/*
 * GMRES-IR driver.  x0 = M^-1 b; then repeat: eta = HPL scaled residual of
 * x; stop when eta < tol; otherwise one GMRES cycle (restart m) on the
 * correction.  Fails (returns 2) if more than max_iters inner iterations
 * would be needed.  Returns 0 on success.  *iters = inner iterations,
 * *cycles = restart cycles, *eta_out = the final scaled residual.
 */
int orc_gmres_ir(int64_t n, const double *A, int64_t lda, const double *P, int64_t ldp, const double *b,
                 double *x, int64_t m, int64_t max_iters, double tol, double tau,
                 int64_t *iters, int64_t *cycles, double *eta_out)
{
    orc_system s = {n, A, lda, P, ldp};
    double *V = (double *)malloc((size_t)n * (size_t)(m + 1) * sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    int64_t it = 0, cyc = 0;
    int status = 0;
    apply_prec(&s, b, x);
    double eta = orc_hpl_eta(n, A, lda, x, b);
    while (!(eta < tol)) {
        if (it >= max_iters) { status = 2; break; }
        int64_t k = orc_gmres_cycle(n, A, lda, P, ldp, b, x, m, tau, &it, max_iters, V, H, NULL, NULL);
        ++cyc;
        eta = orc_hpl_eta(n, A, lda, x, b);
        if (k == 0 && !(eta < tol)) { status = 2; break; } /* no progress possible */
    }
    *iters = it;
    *cycles = cyc;
    *eta_out = eta;
    free(V);
    free(H);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Round-to-nearest-even conversions, from the format definitions            */
/* ------------------------------------------------------------------------ */

/*
 * Format table: p = significand bits including the hidden bit, emin = the
 * exponent of the smallest normal number, maxval = largest finite value.
 * fmt: 0 = fp32, 1 = fp16, 2 = bf16, 3 = fp8 e4m3fn (OCP, no infinities).
 * Overflow: fp32/fp16/bf16 give +-inf (IEEE); e4m3fn saturates to +-448
 * when sat != 0, else returns NaN.
 */
static void fmt_params(int fmt, int *p, int *emin, double *maxval)
{
    switch (fmt) {
    case 0: *p = 24; *emin = -126; *maxval = ldexp(2.0 - ldexp(1.0, -23), 127); break;
    case 1: *p = 11; *emin = -14; *maxval = 65504.0; break;
    case 2: *p = 8; *emin = -126; *maxval = ldexp(2.0 - ldexp(1.0, -7), 127); break;
    default: *p = 4; *emin = -6; *maxval = 448.0; break;
    }
}

double orc_round_fmt(int fmt, double x, int sat)
{
    int p, emin;
    double maxval;
    fmt_params(fmt, &p, &emin, &maxval);
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(fabs(x), &e);            /* |x| = f 2^e with f in [0.5, 1): exponent e-1 */
    int ex = e - 1;
    if (ex < emin) ex = emin;      /* subnormal range: fixed quantum */
    double q = ldexp(1.0, ex - (p - 1));
    double r = nearbyint(x / q);   /* x / q is exact; default mode is ties-to-even */
    double y = r * q;
    if (fabs(y) > maxval) {
        if (fmt == 3) return sat ? copysign(maxval, x) : NAN;
        /* IEEE overflow: beyond max + half ulp -> inf; exact tie handled by RNE above */
        return copysign(INFINITY, x);
    }
    return y;
}

/* encode a value that is already representable in the format */
uint32_t orc_encode_fmt(int fmt, double y)
{
    if (fmt == 0) { float f = (float)y; uint32_t u; memcpy(&u, &f, 4); return u; }
    int p, emin;
    double maxval;
    fmt_params(fmt, &p, &emin, &maxval);
    int ebits = (fmt == 1) ? 5 : (fmt == 2) ? 8 : 4;
    int bias = (1 << (ebits - 1)) - 1;
    uint32_t sign = signbit(y) ? 1u : 0u;
    uint32_t tot = (uint32_t)(1 + ebits + (p - 1));
    if (isnan(y)) return (fmt == 3) ? ((sign << 7) | 0x7Fu) : ((sign << (tot - 1)) | (((1u << ebits) - 1) << (p - 1)) | 1u);
    if (isinf(y)) return (sign << (tot - 1)) | (((1u << ebits) - 1) << (p - 1));
    double a = fabs(y);
    if (a == 0.0) return sign << (tot - 1);
    int e;
    frexp(a, &e);
    int ex = e - 1;
    uint32_t efield, mfield;
    if (ex < emin) { /* subnormal */
        efield = 0;
        mfield = (uint32_t)ldexp(a, -(emin - (p - 1)));
    } else {
        efield = (uint32_t)(ex + bias);
        mfield = (uint32_t)(ldexp(a, -(ex - (p - 1))) - ldexp(1.0, p - 1));
    }
    return (sign << (tot - 1)) | (efield << (p - 1)) | mfield;
}
