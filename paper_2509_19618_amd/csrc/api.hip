// api.hip -- the extern "C" entry points of libmxp (declared in include/mxp.h).
#include <math.h>
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
static bool valid_kind(int kind) { return kind == MXP_GEN_DOMINANT || kind == MXP_GEN_SQRTN || kind == MXP_GEN_UNIFORM; }

extern "C" int mxp_generate(int64_t n, int64_t nrhs, uint64_t seed, int kind, double gamma, int store, void* A,
                            int64_t lda, double* B, int64_t ldb, double* diag, double* row_l1, double* a_inf,
                            void* stream) {
    if (n < 1 || n >= (1ll << 31) || nrhs < 0) return set_err(MXP_EINVAL, "mxp_generate: bad size%s", "");
    if (!valid_kind(kind) || (kind == MXP_GEN_SQRTN && !(gamma > 0 && gamma < 1e300)))
        return set_err(MXP_EINVAL, "mxp_generate: bad kind/gamma%s", "");
    if (A && (!valid_store(store) || lda < n)) return set_err(MXP_EINVAL, "mxp_generate: bad store/lda%s", "");
    if (!diag || !a_inf) return set_err(MXP_EINVAL, "mxp_generate: diag and a_inf are required%s", "");
    if (nrhs > 0 && (!B || ldb < n)) return set_err(MXP_EINVAL, "mxp_generate: bad B/ldb%s", "");
    // the diagonal shift gamma sqrt(n), rounded once per operation in FP64
    const double shift = kind == MXP_GEN_SQRTN ? gamma * sqrt((double)n) : 0.0;
    HIPCHK(generate(n, nrhs, seed, kind, shift, A ? store : MXP_F32, A, lda, B, ldb, diag, row_l1, a_inf,
                    (hipStream_t)stream));
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

extern "C" int mxp_factor_get_layout(int64_t n, int64_t nb, int update, mxp_factor_layout* out) {
    if (n < 1 || n >= (1ll << 31) || nb < 64 || nb > 1024 || nb % 64 || dtype_bytes(update) == 0 || !out)
        return set_err(MXP_EINVAL, "mxp_factor_get_layout: bad argument%s", "");
    const AuxLayout a = aux_layout(n, nb);
    const WorkLayout w = work_layout(n, nb, update);
    out->T = a.T; out->Trm = a.Trm; out->linv = a.linv; out->uinv = a.uinv; out->lsc = a.lsc;
    out->rowscale = a.rowscale; out->linv_full = a.linv_full; out->uinv_full = a.uinv_full; out->aux_bytes = a.total;
    out->Lq = w.Lq; out->Uq = w.Uq; out->inv_sa = w.inv_sa; out->inv_sb = w.inv_sb; out->info = w.info;
    out->work_bytes = w.total;
    out->op_rows = operand_rows(n);
    out->strips = (n + 31) / 32;
    return MXP_OK;
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
        p.pairw = (float*)(w + wl.pairw);
        p.binv = w + wl.binv;
        p.binv_sc = (float*)(w + wl.binv_sc);
    } else {
        p.Lq = p.Uq = nullptr;
        p.inv_sa = p.inv_sb = nullptr;
        p.info = nullptr;
        p.dsync = nullptr;
        p.pairw = nullptr;
        p.binv = nullptr;
        p.binv_sc = nullptr;
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

extern "C" int mxp_factor_group(int count, const mxp_factor_item* items, int update, int store, int tile,
                                int64_t* info, void* stream) {
    if (count < 1 || count > GEMM_GROUP_MAX || !items || !valid_pair(update, store) ||
        (tile != MXP_TILE_256x128 && tile != MXP_TILE_128x128))
        return set_err(MXP_EINVAL, "mxp_factor_group: bad argument%s", "");
    FactorPlan plans[GEMM_GROUP_MAX];
    for (int g = 0; g < count; ++g) {
        const mxp_factor_item& it = items[g];
        if (it.n < 1 || it.n >= (1ll << 31) || !valid_nb(it.nb, update) || it.lda < it.n || !it.A || !it.aux ||
            !it.work)
            return set_err(MXP_EINVAL, "mxp_factor_group: bad item%s", "");
        if (it.work_bytes < work_layout(it.n, it.nb, update).total)
            return set_err(MXP_EWORKSPACE, "mxp_factor_group: work buffer too small%s", "");
        plans[g] = make_plan(it.n, it.nb, update, store, it.A, it.lda, it.aux, it.work);
        plans[g].gemm_tile = tile == MXP_TILE_128x128 ? GEMM_TILE_128 : GEMM_TILE_256;
    }
    hipStream_t s = (hipStream_t)stream;
    for (int g = 0; g < count; ++g) HIPCHK(fill_f64(plans[g].rowscale, plans[g].n, 1.0, s));
    HIPCHK(factor_group(plans, count, s));
    if (info) {
        unsigned long long v[GEMM_GROUP_MAX];
        for (int g = 0; g < count; ++g) HIPCHK(hipMemcpyAsync(&v[g], plans[g].info, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int rc = MXP_OK;
        for (int g = 0; g < count; ++g) {
            info[g] = (v[g] == ~0ull) ? 0 : (int64_t)v[g];
            if (info[g] == (1ll << 62)) {
                info[g] = 0;
                return set_err(MXP_EHIP, "mxp_factor_group: a wait of the diagonal-block LU expired%s", "");
            }
            if (info[g]) rc = MXP_ESINGULAR;
        }
        return rc;
    }
    return MXP_OK;
}

// ------------------------------------------------------------------ solve
// right-hand sides refined together (in lockstep) by one pass of the solve loop
constexpr int RHS_BATCH = 16;

struct SolveLayout {
    size_t V, W, Rr, Z, P, Wp, part, epart, H, cs, sn, g, y, eta4, beta, xnorm, ints, total;
};
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
static SolveLayout solve_layout(int64_t n, int64_t nrhs, int restart) {
    SolveLayout L;
    size_t off = 0;
    const int m = restart, ldh = restart + 1;
    const int R = (int)std::min<int64_t>(std::max<int64_t>(nrhs, 1), RHS_BATCH);
    L.V = off; off = al256(off + (size_t)n * (m + 1) * R * 8);
    L.W = off; off = al256(off + (size_t)n * R * 8);
    L.Rr = off; off = al256(off + (size_t)n * R * 8);
    L.Z = off; off = al256(off + (size_t)n * R * 8);
    L.P = off; off = al256(off + regen_partial_bytes(n, R < 8 ? R : 8));
    L.Wp = off; off = al256(off + prec_work_bytes(n, R));
    L.part = off; off = al256(off + (size_t)2 * R * 256 * 8);
    L.epart = off; off = al256(off + (size_t)eta_blocks(n) * 3 * R * 8);
    L.H = off; off = al256(off + (size_t)R * ldh * m * 8);
    L.cs = off; off = al256(off + (size_t)R * ldh * 8);
    L.sn = off; off = al256(off + (size_t)R * ldh * 8);
    L.g = off; off = al256(off + (size_t)R * ldh * 8);
    L.y = off; off = al256(off + (size_t)R * ldh * 8);
    L.eta4 = off; off = al256(off + (size_t)R * 4 * 8);
    L.beta = off; off = al256(off + (size_t)R * 8);
    L.xnorm = off; off = al256(off + (size_t)R * 8);
    L.ints = off; off = al256(off + (size_t)3 * RHS_BATCH * 4);
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

// per-right-hand-side integers handed to the device as a launch argument
struct IntVec {
    int v[RHS_BATCH];
};
__global__ void k_set_ints(int* dst, int n, IntVec vals) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = vals.v[threadIdx.x];
}

// GMRES-IR for up to RHS_BATCH right-hand sides at once: every matrix product
// and preconditioner apply serves all of them in one launch, the vector
// steps run per right-hand side in the same launches, and the host reads the
// convergence scalars of all of them with one synchronisation per step.
static int solve_batch(int64_t n, uint64_t seed, int kind, const PrecPlan& pp, const double* diag, const double* a_inf,
                       const double* B, int64_t ldb, double* X, int64_t ldx, int R, int restart, int max_iters,
                       double tol, double tau, mxp_rhs_report* rep, char* wb, const SolveLayout& L, hipStream_t s) {
    double* V = (double*)(wb + L.V);
    double* W = (double*)(wb + L.W);
    double* Rr = (double*)(wb + L.Rr);
    double* Z = (double*)(wb + L.Z);
    double* P = (double*)(wb + L.P);
    double* Wp = (double*)(wb + L.Wp);
    double* part = (double*)(wb + L.part);
    double* epart = (double*)(wb + L.epart);
    double* H = (double*)(wb + L.H);
    double* cs = (double*)(wb + L.cs);
    double* sn = (double*)(wb + L.sn);
    double* g = (double*)(wb + L.g);
    double* y = (double*)(wb + L.y);
    double* eta4 = (double*)(wb + L.eta4);
    double* beta = (double*)(wb + L.beta);
    double* xnorm = (double*)(wb + L.xnorm);
    int* act = (int*)(wb + L.ints);
    int* flag = act + RHS_BATCH;
    int* kdim = flag + RHS_BATCH;
    const int m = restart, ldh = restart + 1;
    auto upload = [&](int* dst, const int* v) -> hipError_t {
        IntVec iv;
        for (int r = 0; r < RHS_BATCH; ++r) iv.v[r] = r < R ? v[r] : 0;
        k_set_ints<<<1, 64, 0, s>>>(dst, R, iv);
        return hipGetLastError();
    };
    int64_t it[RHS_BATCH] = {}, cyc[RHS_BATCH] = {};
    int status[RHS_BATCH], done[RHS_BATCH] = {}, a[RHS_BATCH], kd[RHS_BATCH];
    double eta[RHS_BATCH] = {};
    for (int r = 0; r < R; ++r) status[r] = MXP_OK;
    HIPCHK(prec_apply(pp, B, ldb, X, ldx, R, Wp, s));   // x0 = M^-1 b
    for (;;) {
        HIPCHK(regen_matvec(n, seed, kind, diag, X, ldx, R, B, ldb, Rr, n, P, s));
        HIPCHK(hpl_eta_dev(n, R, Rr, n, X, ldx, B, ldb, a_inf, epart, eta4, s));
        double eh[4 * RHS_BATCH];
        HIPCHK(hipMemcpyAsync(eh, eta4, (size_t)4 * R * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int nact = 0;
        for (int r = 0; r < R; ++r) {
            a[r] = 0;
            if (done[r]) continue;
            eta[r] = eh[4 * r];
            if (eta[r] < tol) { done[r] = 1; continue; }
            if (it[r] >= max_iters || !(eta[r] == eta[r])) { status[r] = MXP_ENOCONV; done[r] = 1; continue; }
            a[r] = 1;
            ++nact;
        }
        if (!nact) break;
        HIPCHK(upload(act, a));
        // z = M^-1 r ; beta = ||z|| ; v0 = z / beta ; g = beta e1 ; ||x||
        HIPCHK(prec_apply(pp, Rr, n, Z, n, R, Wp, s));
        HIPCHK(gm_norms(n, R, Z, n, beta, 1, part, act, s));
        HIPCHK(gm_start(n, R, Z, beta, 1, V, g, ldh, act, s));
        HIPCHK(gm_norms(n, R, X, ldx, xnorm, 1, part, act, s));
        int in[RHS_BATCH];
        for (int r = 0; r < R; ++r) { in[r] = a[r]; kd[r] = 0; }
        for (int j = 0; j < m; ++j) {
            int nin = 0;
            for (int r = 0; r < R; ++r) {
                if (in[r] && it[r] >= max_iters) in[r] = 0;
                nin += in[r];
            }
            if (!nin) break;
            if (j > 0) HIPCHK(upload(act, in));
            for (int r = 0; r < R; ++r)
                if (in[r]) { ++it[r]; kd[r] = j + 1; }
            // w = M^-1 A v_j for every right-hand side
            HIPCHK(regen_matvec(n, seed, kind, diag, V + (int64_t)j * R * n, n, R, nullptr, n, W, n, P, s));
            HIPCHK(prec_apply(pp, W, n, W, n, R, Wp, s));
            HIPCHK(gm_arnoldi(n, R, V, j, W, part, H, ldh, act, s));
            HIPCHK(gm_givens(R, j, H, ldh, cs, sn, g, xnorm, 1, tau, flag, act, s));
            int fl[RHS_BATCH];
            HIPCHK(hipMemcpyAsync(fl, flag, (size_t)R * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int r = 0; r < R; ++r)
                if (in[r] && fl[r]) in[r] = 0;
        }
        HIPCHK(upload(kdim, kd));
        HIPCHK(gm_update(n, R, H, ldh, g, y, kdim, V, X, ldx, s));
        for (int r = 0; r < R; ++r) {
            if (!a[r]) continue;
            ++cyc[r];
            if (kd[r] == 0) { status[r] = MXP_ENOCONV; done[r] = 1; }
        }
    }
    int worst = MXP_OK;
    for (int r = 0; r < R; ++r) {
        if (status[r] == MXP_OK && !(eta[r] < tol)) status[r] = MXP_ECRITERION;
        rep[r].iters = it[r];
        rep[r].cycles = cyc[r];
        rep[r].eta = eta[r];
        rep[r].status = status[r];
        rep[r].pad = 0;
        if (status[r] > worst) worst = status[r];
    }
    return worst;
}

extern "C" int mxp_solve_ir(int64_t n, int64_t nb, int update, int store, uint64_t seed, int kind, const void* LU,
                            int64_t lda, const void* aux, const double* diag, const double* a_inf, const double* B,
                            int64_t ldb, double* X, int64_t ldx, int64_t nrhs, int restart, int max_iters, double tol,
                            double tau, mxp_rhs_report* rep, void* work, size_t work_bytes, void* stream) {
    if (n < 1 || n >= (1ll << 31) || !valid_pair(update, store) || !valid_nb(nb, update) || lda < n || !LU || !aux ||
        !valid_kind(kind) || !diag || !a_inf || !B || !X || ldb < n || ldx < n || nrhs < 1 || restart < 1 ||
        restart > 64 || max_iters < 1 || !(tol > 0) || !(tau >= 0) || !rep || !work)
        return set_err(MXP_EINVAL, "mxp_solve_ir: bad argument%s", "");
    SolveLayout L = solve_layout(n, nrhs, restart);
    if (work_bytes < L.total) return set_err(MXP_EWORKSPACE, "mxp_solve_ir: work buffer too small%s", "");
    hipStream_t s = (hipStream_t)stream;
    PrecPlan pp = make_prec(n, nb, store, LU, lda, aux);
    const int Rmax = (int)std::min<int64_t>(nrhs, RHS_BATCH);
    double* Wp = (double*)((char*)work + L.Wp);
    HIPCHK(prec_err_reset(Wp, n, Rmax, s));
    int worst = MXP_OK;
    for (int64_t r0 = 0; r0 < nrhs; r0 += RHS_BATCH) {
        const int R = (int)std::min<int64_t>(nrhs - r0, RHS_BATCH);
        const int rc = solve_batch(n, seed, kind, pp, diag, a_inf, B + r0 * ldb, ldb, X + r0 * ldx, ldx, R, restart,
                                   max_iters, tol, tau, rep + r0, (char*)work, L, s);
        if (rc < 0) return rc;
        if (rc > worst) worst = rc;
    }
    int perr = 0;
    HIPCHK(prec_err_read(Wp, n, Rmax, &perr, s));
    if (perr) return set_err(MXP_EHIP, "mxp_solve_ir: a wait of the block substitution expired%s", "");
    return worst;
}

// ------------------------------------------------------------------ building blocks
extern "C" size_t mxp_residual_work_bytes(int64_t n, int64_t nrhs) {
    if (n < 1 || nrhs < 1) return 0;
    return regen_partial_bytes(n, nrhs < 8 ? (int)nrhs : 8);
}

extern "C" int mxp_residual(int64_t n, uint64_t seed, int kind, const double* diag, const double* X, int64_t ldx,
                            const double* B, int64_t ldb, double* R, int64_t ldr, int64_t nrhs, void* work,
                            size_t work_bytes, void* stream) {
    if (n < 1 || n >= (1ll << 31) || nrhs < 1 || !valid_kind(kind) || !diag || !X || !R || ldx < n || ldr < n ||
        (B && ldb < n) || !work)
        return set_err(MXP_EINVAL, "mxp_residual: bad argument%s", "");
    if (work_bytes < mxp_residual_work_bytes(n, nrhs))
        return set_err(MXP_EWORKSPACE, "mxp_residual: work buffer too small%s", "");
    HIPCHK(regen_matvec(n, seed, kind, diag, X, ldx, (int)nrhs, B, ldb, R, ldr, (double*)work, (hipStream_t)stream));
    return MXP_OK;
}

extern "C" int mxp_residual_noalloc(int64_t n, uint64_t seed, int kind, const double* diag, const double* X,
                                    int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr, int64_t nrhs,
                                    void* stream) {
    if (n < 1 || n >= (1ll << 31) || nrhs < 1 || !valid_kind(kind) || !diag || !X || !R || ldx < n || ldr < n ||
        (B && ldb < n))
        return set_err(MXP_EINVAL, "mxp_residual_noalloc: bad argument%s", "");
    if (mxp_residual_work_bytes(n, nrhs) > static_scratch_bytes())
        return set_err(MXP_EINVAL, "mxp_residual_noalloc: n * min(nrhs, 8) too large for the library's %s scratch",
                       "32 MiB");
    void* scr = nullptr;
    HIPCHK(static_scratch(&scr));
    HIPCHK(regen_matvec(n, seed, kind, diag, X, ldx, (int)nrhs, B, ldb, R, ldr, (double*)scr, (hipStream_t)stream));
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

extern "C" int mxp_hpl_eta(int64_t n, uint64_t seed, int kind, const double* diag, const double* a_inf,
                           const double* x, const double* b, double* eta, void* work, size_t work_bytes,
                           void* stream) {
    if (n < 1 || n >= (1ll << 31) || !valid_kind(kind) || !diag || !a_inf || !x || !b || !eta || !work)
        return set_err(MXP_EINVAL, "mxp_hpl_eta: bad argument%s", "");
    if (work_bytes < mxp_hpl_eta_work_bytes(n)) return set_err(MXP_EWORKSPACE, "mxp_hpl_eta: work too small%s", "");
    hipStream_t s = (hipStream_t)stream;
    char* wb = (char*)work;
    double* P = (double*)wb;
    double* r = (double*)(wb + regen_partial_bytes(n, 1));
    double* ep = (double*)((char*)r + al256((size_t)n * 8));
    double* out = (double*)((char*)ep + al256(3 * 512 * 8));
    HIPCHK(regen_matvec(n, seed, kind, diag, x, n, 1, b, n, r, n, P, s));
    HIPCHK(hpl_eta_dev(n, 1, r, n, x, n, b, n, a_inf, ep, out, s));
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

extern "C" int mxp_trailing_update2(int64_t M, int64_t N, int64_t K1, int64_t K2, int update, int store, void* C,
                                    int64_t ldc, const void* Aq1, const void* Bq1, const float* inv_sa1,
                                    const float* inv_sb1, const void* Aq2, const void* Bq2, const float* inv_sa2,
                                    const float* inv_sb2, void* stream) {
    if (M < 0 || N < 0 || K1 < 1 || K1 > 4096 || K2 < 1 || K2 > 4096 || ldc < (M > 1 ? M : 1) ||
        !valid_pair(update, store) || (K1 * dtype_bytes(update)) % 128 || (K2 * dtype_bytes(update)) % 128 ||
        (M > 0 && N > 0 && (!C || !Aq1 || !Bq1 || !inv_sa1 || !inv_sb1 || !Aq2 || !Bq2 || !inv_sa2 || !inv_sb2)))
        return set_err(MXP_EINVAL, "mxp_trailing_update2: bad argument%s", "");
    if (M == 0 || N == 0) return MXP_OK;
    GemmCall c{C, ldc, M, N, (int)K1, Aq1, Bq1, inv_sa1, inv_sb1};
    c.K2 = (int)K2;
    c.Aq2 = Aq2; c.Bq2 = Bq2; c.inv_sa2 = inv_sa2; c.inv_sb2 = inv_sb2;
    hipEvent_t pt = prof::begin(prof::GEMM, (hipStream_t)stream);
    HIPCHK(gemm_group(update, store, GEMM_TILE_256, &c, 1, (hipStream_t)stream));
    prof::end(pt, prof::GEMM, (hipStream_t)stream, 2.0 * M * (double)N * (K1 + K2),
              2.0 * M * (double)N * dtype_bytes(store) + (double)(M + N) * (K1 + K2) * dtype_bytes(update));
    return MXP_OK;
}

// ------------------------------------------------------------------ FP64 LU
extern "C" size_t mxp_lu64_work_bytes(int64_t n) {
    if (n < 1 || n >= (1ll << 31)) return 0;
    return lu64_work_bytes(n) + 256;
}

extern "C" int mxp_lu64_factor(int64_t n, double* A, int64_t lda, int64_t* ipiv, int gemm, void* work,
                               size_t work_bytes, int64_t* info, void* stream) {
    if (n < 1 || n >= (1ll << 31) || !A || lda < n || !work || (ipiv && n > 65536) ||
        (gemm != MXP_GEMM64_OWN && gemm != MXP_GEMM64_ROCBLAS))
        return set_err(MXP_EINVAL, "mxp_lu64_factor: bad argument%s", "");
    if (work_bytes < mxp_lu64_work_bytes(n)) return set_err(MXP_EWORKSPACE, "mxp_lu64_factor: work too small%s", "");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* info_dev = (unsigned long long*)((char*)work + lu64_work_bytes(n));
    HIPCHK(lu64_factor(n, A, lda, ipiv, work, info_dev, gemm == MXP_GEMM64_ROCBLAS, s));
    if (info) {
        unsigned long long v = 0;
        int err = 0;
        HIPCHK(hipMemcpyAsync(&v, info_dev, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&err, lu64_err_word(work, n), 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (err) return set_err(MXP_EHIP, "mxp_lu64_factor: a grid barrier of the pivoted panel expired%s", "");
        *info = (v == ~0ull) ? 0 : (int64_t)v;
        if (*info) return MXP_ESINGULAR;
    }
    return MXP_OK;
}

extern "C" int mxp_lu64_solve(int64_t n, const double* LU, int64_t lda, const int64_t* ipiv, double* X, int64_t ldx,
                              int64_t nrhs, void* stream) {
    if (n < 1 || n >= (1ll << 31) || !LU || lda < n || !X || ldx < n || nrhs < 1 || nrhs > 64)
        return set_err(MXP_EINVAL, "mxp_lu64_solve: bad argument%s", "");
    HIPCHK(lu64_solve(n, LU, lda, ipiv, X, ldx, (int)nrhs, (hipStream_t)stream));
    return MXP_OK;
}

extern "C" int mxp_trailing_update64(int64_t M, int64_t N, int64_t K, double* C, int64_t ldc, const double* A,
                                     int64_t lda, const double* B, int64_t ldb, void* stream) {
    if (M < 0 || N < 0 || K < 1 || K % 4 || ldc < (M > 1 ? M : 1) || lda < (M > 1 ? M : 1) || ldb < K ||
        (M > 0 && N > 0 && (!C || !A || !B)))
        return set_err(MXP_EINVAL, "mxp_trailing_update64: bad argument%s", "");
    HIPCHK(gemm64(C, ldc, A, lda, B, ldb, M, N, (int)K, (hipStream_t)stream));
    return MXP_OK;
}
