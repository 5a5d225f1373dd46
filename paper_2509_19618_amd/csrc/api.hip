// api.hip -- the extern "C" entry points of libmxp (declared in include/mxp.h).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/mxp.h"
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

using namespace mxp;

static thread_local char g_err[512] = "";

static int set_err(int code, const char* fmt, const char* what) {
    snprintf(g_err, sizeof(g_err), fmt, what);
    return code;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) {                                                               \
            snprintf(g_err, sizeof(g_err), "%s: %s", #expr, hipGetErrorString(_e));           \
            return MXP_EHIP;                                                                  \
        }                                                                                     \
    } while (0)

extern "C" const char* mxp_last_error(void) { return g_err; }
extern "C" const char* mxp_version(void) { return "libmxp 0.1 (gfx950)"; }

static bool valid_store(int st) { return st == MXP_F64 || st == MXP_F32 || st == MXP_F16 || st == MXP_BF16; }
static bool valid_pair(int update, int store) {
    return (update == MXP_F32 && store == MXP_F32) || (update == MXP_F16 && store == MXP_F16) ||
           (update == MXP_BF16 && store == MXP_BF16) || (update == MXP_F8E4M3 && store == MXP_F16) ||
           (update == MXP_F8E4M3 && store == MXP_BF16) || (update == MXP_F16 && store == MXP_F32) ||
           (update == MXP_BF16 && store == MXP_F32);
}
static bool valid_nb(int64_t nb, int update) {
    if (nb < 64 || nb > 1024 || nb % 64) return false;
    if (update == MXP_F8E4M3 && nb % 128) return false;
    return true;
}

// ------------------------------------------------------------------ generate
extern "C" int mxp_generate(int64_t n, int64_t nrhs, uint64_t seed, int store, void* A, int64_t lda, double* B,
                            int64_t ldb, double* diag, double* a_inf, void* stream) {
    if (n < 1 || n >= (1ll << 31) || nrhs < 0) return set_err(MXP_EINVAL, "mxp_generate: bad size%s", "");
    if (A && (!valid_store(store) || lda < n)) return set_err(MXP_EINVAL, "mxp_generate: bad store/lda%s", "");
    if (!diag || !a_inf) return set_err(MXP_EINVAL, "mxp_generate: diag and a_inf are required%s", "");
    if (nrhs > 0 && (!B || ldb < n)) return set_err(MXP_EINVAL, "mxp_generate: bad B/ldb%s", "");
    HIPCHK(generate(n, nrhs, seed, A ? store : MXP_F32, A, lda, B, ldb, diag, a_inf, (hipStream_t)stream));
    return MXP_OK;
}

// ------------------------------------------------------------------ factor
extern "C" size_t mxp_factor_aux_bytes(int64_t n, int64_t nb) {
    if (n < 1 || nb < 64) return 0;
    return aux_layout(n, nb).total;
}

extern "C" size_t mxp_factor_work_bytes(int64_t n, int64_t nb, int update) {
    if (n < 1 || nb < 64 || dtype_bytes(update) == 0) return 0;
    return work_layout(n, nb, update).total;
}

static FactorPlan make_plan(int64_t n, int64_t nb, int update, int store, void* A, int64_t lda, void* aux,
                            void* work) {
    FactorPlan p;
    p.n = n; p.nb = nb; p.lda = lda; p.update = update; p.store = store; p.A = A;
    p.op_rows = operand_rows(n);
    AuxLayout al = aux_layout(n, nb);
    char* a = (char*)aux;
    p.T = (float*)(a + al.T);
    p.Trm = (float*)(a + al.Trm);
    p.linv = (float*)(a + al.linv);
    p.uinv = (float*)(a + al.uinv);
    p.lsc = (float*)(a + al.lsc);
    p.rowscale = (double*)(a + al.rowscale);
    p.linv_full = (float*)(a + al.linv_full);
    p.uinv_full = (float*)(a + al.uinv_full);
    if (work) {
        WorkLayout wl = work_layout(n, nb, update);
        char* w = (char*)work;
        p.Lq = w + wl.Lq;
        p.Uq = w + wl.Uq;
        p.inv_sa = (float*)(w + wl.inv_sa);
        p.inv_sb = (float*)(w + wl.inv_sb);
        p.info = (unsigned long long*)(w + wl.info);
        p.dsync = (int*)(w + wl.dsync);
    } else {
        p.Lq = p.Uq = nullptr;
        p.inv_sa = p.inv_sb = nullptr;
        p.info = nullptr;
        p.dsync = nullptr;
    }
    return p;
}

__global__ void k_fill_scalar_f64(double* p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

static hipError_t fill_f64(double* p, int64_t n, double v, hipStream_t s) {
    k_fill_scalar_f64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

namespace mxp {
int factor_with(int64_t n, int64_t nb, int update, int store, int scaling, const double* diag, void* A, int64_t lda,
                void* aux, void* work, size_t work_bytes, int64_t* info, hipStream_t s, Lookahead* la) {
    if (n < 1 || n >= (1ll << 31) || !valid_pair(update, store) || !valid_nb(nb, update) || lda < n || !A || !aux ||
        !work || (scaling != MXP_SCALE_NONE && scaling != MXP_SCALE_ROW_EQUIL) ||
        (scaling == MXP_SCALE_ROW_EQUIL && !diag))
        return set_err(MXP_EINVAL, "mxp_factor: bad argument%s", "");
    if (work_bytes < work_layout(n, nb, update).total)
        return set_err(MXP_EWORKSPACE, "mxp_factor: work buffer too small%s", "");
    FactorPlan p = make_plan(n, nb, update, store, A, lda, aux, work);
    if (scaling == MXP_SCALE_ROW_EQUIL) HIPCHK(row_equilibrate(p, diag, s));
    else HIPCHK(fill_f64(p.rowscale, n, 1.0, s));
    HIPCHK(factor_run(p, s, la));
    if (info) {
        unsigned long long v = 0;
        HIPCHK(hipMemcpyAsync(&v, p.info, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *info = (v == ~0ull) ? 0 : (int64_t)v;
        if (*info == (1ll << 62)) {
            *info = 0;
            return set_err(MXP_EHIP, "mxp_factor: a wait of the diagonal-block LU expired%s", "");
        }
        if (*info) return MXP_ESINGULAR;
    }
    return MXP_OK;
}
}  // namespace mxp

extern "C" int mxp_factor(int64_t n, int64_t nb, int update, int store, int scaling, const double* diag, void* A,
                          int64_t lda, void* aux, void* work, size_t work_bytes, int64_t* info, void* stream) {
    return factor_with(n, nb, update, store, scaling, diag, A, lda, aux, work, work_bytes, info, (hipStream_t)stream,
                       nullptr);
}

// ------------------------------------------------------------------ solve
struct SolveLayout {
    size_t V, w, r, z, P, W, part, epart, H, cs, sn, g, y, sc, total;
};
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
static SolveLayout solve_layout(int64_t n, int64_t nrhs, int restart) {
    SolveLayout L;
    size_t off = 0;
    int m = restart;
    L.V = off; off = al256(off + (size_t)n * (m + 1) * 8);
    L.w = off; off = al256(off + (size_t)n * 8);
    L.r = off; off = al256(off + (size_t)n * 8);
    L.z = off; off = al256(off + (size_t)n * 8);
    L.P = off; off = al256(off + regen_partial_bytes(n, 8 < nrhs ? 8 : (int)std::max<int64_t>(nrhs, 1)));
    L.W = off; off = al256(off + prec_work_bytes(n, 1));
    L.part = off; off = al256(off + 2 * 256 * 8);
    L.epart = off; off = al256(off + 3 * 512 * 8);
    L.H = off; off = al256(off + (size_t)(m + 1) * m * 8);
    L.cs = off; off = al256(off + (size_t)(m + 1) * 8);
    L.sn = off; off = al256(off + (size_t)(m + 1) * 8);
    L.g = off; off = al256(off + (size_t)(m + 1) * 8);
    L.y = off; off = al256(off + (size_t)(m + 1) * 8);
    L.sc = off; off = al256(off + 16 * 8);
    L.total = off;
    return L;
}

extern "C" size_t mxp_solve_work_bytes(int64_t n, int64_t nrhs, int restart) {
    if (n < 1 || nrhs < 0 || restart < 1 || restart > 64) return 0;
    return solve_layout(n, nrhs, restart).total;
}

static PrecPlan make_prec(int64_t n, int64_t nb, int store, const void* LU, int64_t lda, const void* aux) {
    FactorPlan f = make_plan(n, nb, MXP_F32, store, (void*)LU, lda, (void*)aux, nullptr);
    PrecPlan p;
    p.n = n; p.nb = nb; p.lda = lda; p.store = store; p.A = LU;
    p.T = f.T; p.linv = f.linv; p.uinv = f.uinv; p.lsc = f.lsc; p.rowscale = f.rowscale;
    p.linv_full = f.linv_full; p.uinv_full = f.uinv_full;
    return p;
}

extern "C" int mxp_solve_ir(int64_t n, int64_t nb, int update, int store, uint64_t seed, const void* LU, int64_t lda,
                            const void* aux, const double* diag, const double* a_inf, const double* B, int64_t ldb,
                            double* X, int64_t ldx, int64_t nrhs, int restart, int max_iters, double tol, double tau,
                            mxp_rhs_report* rep, void* work, size_t work_bytes, void* stream) {
    if (n < 1 || n >= (1ll << 31) || !valid_pair(update, store) || !valid_nb(nb, update) || lda < n || !LU || !aux ||
        !diag || !a_inf || !B || !X || ldb < n || ldx < n || nrhs < 1 || restart < 1 || restart > 64 ||
        max_iters < 1 || !(tol > 0) || !(tau >= 0) || !rep || !work)
        return set_err(MXP_EINVAL, "mxp_solve_ir: bad argument%s", "");
    SolveLayout L = solve_layout(n, nrhs, restart);
    if (work_bytes < L.total) return set_err(MXP_EWORKSPACE, "mxp_solve_ir: work buffer too small%s", "");
    hipStream_t s = (hipStream_t)stream;
    char* wb = (char*)work;
    double* V = (double*)(wb + L.V);
    double* w = (double*)(wb + L.w);
    double* r = (double*)(wb + L.r);
    double* z = (double*)(wb + L.z);
    double* P = (double*)(wb + L.P);
    double* W = (double*)(wb + L.W);
    double* part = (double*)(wb + L.part);
    double* epart = (double*)(wb + L.epart);
    double* H = (double*)(wb + L.H);
    double* cs = (double*)(wb + L.cs);
    double* sn = (double*)(wb + L.sn);
    double* g = (double*)(wb + L.g);
    double* y = (double*)(wb + L.y);
    double* sc = (double*)(wb + L.sc);  // [0..2] eta out, [4] beta, [5] xnorm, [6..7] flag
    const int m = restart, ldh = restart + 1;
    PrecPlan pp = make_prec(n, nb, store, LU, lda, aux);
    HIPCHK(prec_err_reset(W, n, 1, s));
    int worst = MXP_OK;
    for (int64_t rr = 0; rr < nrhs; ++rr) {
        const double* b = B + rr * ldb;
        double* x = X + rr * ldx;
        HIPCHK(prec_apply(pp, b, n, x, n, 1, W, s));  // x0 = M^-1 b
        int64_t it = 0, cyc = 0;
        int status = MXP_OK;
        double eta = 0;
        for (;;) {
            HIPCHK(regen_matvec(n, seed, diag, x, n, 1, b, n, r, n, P, s));
            HIPCHK(hpl_eta_dev(n, r, x, b, a_inf, epart, sc, s));
            double eh[3];
            HIPCHK(hipMemcpyAsync(eh, sc, 3 * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            eta = eh[0];
            if (eta < tol) break;
            if (it >= max_iters || !(eta == eta)) { status = MXP_ENOCONV; break; }
            // z = M^-1 r ; beta = ||z|| ; v0 = z / beta ; g = beta e1
            HIPCHK(prec_apply(pp, r, n, z, n, 1, W, s));
            HIPCHK(fill_f64(g, m + 1, 0.0, s));
            HIPCHK(vec_norm2(n, z, sc + 4, part, s));
            HIPCHK(vec_scale_copy(n, z, sc + 4, V, g, s));
            HIPCHK(vec_norm2(n, x, sc + 5, part, s));
            int kdim = 0;
            for (int j = 0; j < m; ++j) {
                if (it >= max_iters) break;
                ++it;
                HIPCHK(regen_matvec(n, seed, diag, V + (int64_t)j * n, n, 1, nullptr, n, r, n, P, s));
                HIPCHK(prec_apply(pp, r, n, w, n, 1, W, s));
                HIPCHK(mgs_step(n, V, j, w, H + (int64_t)j * ldh, part, s));
                HIPCHK(norm_normalize(n, w, V + (int64_t)(j + 1) * n, H + (int64_t)j * ldh + j + 1,
                                      part + ((j + 1) & 1) * 256, s));
                HIPCHK(givens_step(j, H, ldh, cs, sn, g, sc + 5, tau, sc + 6, s));
                kdim = j + 1;
                double fl[2];
                HIPCHK(hipMemcpyAsync(fl, sc + 6, 16, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                if (fl[1] != 0.0) break;
            }
            HIPCHK(lsq_update(n, kdim, H, ldh, g, y, V, x, s));
            ++cyc;
            if (kdim == 0) { status = MXP_ENOCONV; break; }
        }
        if (status == MXP_OK && !(eta < tol)) status = MXP_ECRITERION;
        rep[rr].iters = it;
        rep[rr].cycles = cyc;
        rep[rr].eta = eta;
        rep[rr].status = status;
        rep[rr].pad = 0;
        if (status > worst) worst = status;
    }
    int perr = 0;
    HIPCHK(prec_err_read(W, n, 1, &perr, s));
    if (perr) return set_err(MXP_EHIP, "mxp_solve_ir: a wait of the block substitution expired%s", "");
    return worst;
}

// ------------------------------------------------------------------ building blocks
extern "C" size_t mxp_residual_work_bytes(int64_t n, int64_t nrhs) {
    if (n < 1 || nrhs < 1) return 0;
    return regen_partial_bytes(n, nrhs < 8 ? (int)nrhs : 8);
}

extern "C" int mxp_residual(int64_t n, uint64_t seed, const double* diag, const double* X, int64_t ldx,
                            const double* B, int64_t ldb, double* R, int64_t ldr, int64_t nrhs, void* work,
                            size_t work_bytes, void* stream) {
    if (n < 1 || n >= (1ll << 31) || nrhs < 1 || !diag || !X || !R || ldx < n || ldr < n || (B && ldb < n) || !work)
        return set_err(MXP_EINVAL, "mxp_residual: bad argument%s", "");
    if (work_bytes < mxp_residual_work_bytes(n, nrhs))
        return set_err(MXP_EWORKSPACE, "mxp_residual: work buffer too small%s", "");
    HIPCHK(regen_matvec(n, seed, diag, X, ldx, (int)nrhs, B, ldb, R, ldr, (double*)work, (hipStream_t)stream));
    return MXP_OK;
}

extern "C" size_t mxp_apply_prec_work_bytes(int64_t n, int64_t nrhs) {
    if (n < 1 || nrhs < 1 || nrhs > 64) return 0;
    return prec_work_bytes(n, (int)nrhs);
}

extern "C" int mxp_apply_prec(int64_t n, int64_t nb, int update, int store, const void* LU, int64_t lda,
                              const void* aux, const double* V, int64_t ldv, double* Z, int64_t ldz, int64_t nrhs,
                              void* work, size_t work_bytes, void* stream) {
    if (n < 1 || n >= (1ll << 31) || !valid_pair(update, store) || !valid_nb(nb, update) || lda < n || !LU || !aux ||
        !V || !Z || ldv < n || ldz < n || nrhs < 1 || nrhs > 64 || !work)
        return set_err(MXP_EINVAL, "mxp_apply_prec: bad argument%s", "");
    if (work_bytes < mxp_apply_prec_work_bytes(n, nrhs))
        return set_err(MXP_EWORKSPACE, "mxp_apply_prec: work buffer too small%s", "");
    PrecPlan pp = make_prec(n, nb, store, LU, lda, aux);
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(prec_err_reset((double*)work, n, (int)nrhs, s));
    HIPCHK(prec_apply(pp, V, ldv, Z, ldz, (int)nrhs, (double*)work, s));
    int perr = 0;
    HIPCHK(prec_err_read((double*)work, n, (int)nrhs, &perr, s));
    if (perr) return set_err(MXP_EHIP, "mxp_apply_prec: a wait of the block substitution expired%s", "");
    return MXP_OK;
}

extern "C" size_t mxp_hpl_eta_work_bytes(int64_t n) {
    if (n < 1) return 0;
    return regen_partial_bytes(n, 1) + al256((size_t)n * 8) + al256(3 * 512 * 8) + 256;
}

extern "C" int mxp_hpl_eta(int64_t n, uint64_t seed, const double* diag, const double* a_inf, const double* x,
                           const double* b, double* eta, void* work, size_t work_bytes, void* stream) {
    if (n < 1 || n >= (1ll << 31) || !diag || !a_inf || !x || !b || !eta || !work)
        return set_err(MXP_EINVAL, "mxp_hpl_eta: bad argument%s", "");
    if (work_bytes < mxp_hpl_eta_work_bytes(n)) return set_err(MXP_EWORKSPACE, "mxp_hpl_eta: work too small%s", "");
    hipStream_t s = (hipStream_t)stream;
    char* wb = (char*)work;
    double* P = (double*)wb;
    double* r = (double*)(wb + regen_partial_bytes(n, 1));
    double* ep = (double*)((char*)r + al256((size_t)n * 8));
    double* out = (double*)((char*)ep + al256(3 * 512 * 8));
    HIPCHK(regen_matvec(n, seed, diag, x, n, 1, b, n, r, n, P, s));
    HIPCHK(hpl_eta_dev(n, r, x, b, a_inf, ep, out, s));
    HIPCHK(hipMemcpyAsync(eta, out, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MXP_OK;
}

extern "C" int mxp_trailing_update(int64_t M, int64_t N, int64_t K, int update, int store, void* C, int64_t ldc,
                                   const void* Aq, const void* Bq, const float* inv_sa, const float* inv_sb,
                                   void* stream) {
    if (M < 0 || N < 0 || K < 1 || K > 4096 || ldc < (M > 1 ? M : 1) || !valid_pair(update, store) ||
        (K * dtype_bytes(update)) % 128 || (M > 0 && N > 0 && (!C || !Aq || !Bq || !inv_sa || !inv_sb)))
        return set_err(MXP_EINVAL, "mxp_trailing_update: bad argument%s", "");
    hipEvent_t pt = prof::begin(prof::GEMM, (hipStream_t)stream);
    HIPCHK(gemm_update(update, store, C, ldc, M, N, (int)K, Aq, Bq, inv_sa, inv_sb, (hipStream_t)stream));
    prof::end(pt, prof::GEMM, (hipStream_t)stream, 2.0 * M * (double)N * K,
              2.0 * M * (double)N * dtype_bytes(store) + (double)(M + N) * K * dtype_bytes(update));
    return MXP_OK;
}
