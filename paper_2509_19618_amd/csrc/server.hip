// server.hip -- continuous-batching solve server on one device (host runtime).
//
// Every request (n, nrhs, seed) runs the same path as a direct call of
// mxp_generate + mxp_factor + mxp_solve_ir (the paper's statement of the
// problem: a generated, diagonally dominant system solved by low-precision
// LU and FP64 GMRES-IR to the HPL backward-error test).  The server adds:
//
//   * admission by HBM budget: the caller's arena is sub-allocated first-fit
//     (256-byte granules); the request at the head of the queue is admitted
//     as soon as a slot is idle and its bytes fit, so requests arriving while
//     others run start as slots and memory free up (arrival order is kept,
//     which bounds the wait of large requests);
//   * workers: a few host threads (at most three, fewer than the device's four
//     hardware queues), each with one stream.  A worker takes a group of up
//     to eight admitted requests and factors them together: per block step
//     ONE launch of the diagonal-block LU, ONE of the strip TRSMs and ONE of
//     the trailing update serve the whole group through descriptor arrays
//     (mxp_factor_group).  It then refines each request with all of its
//     right-hand sides in lockstep (mxp_solve_ir) and hands it back as soon
//     as its own refinement ends.  The workers' groups overlap on the device;
//   * a tuner: per size class (powers of two 512 .. 16384) it times every
//     candidate pair of block size and trailing-update tile at creation and
//     keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "mxp.h"

namespace mxp {
namespace {

constexpr size_t GRAN = 256;
size_t al(size_t x) { return (x + GRAN - 1) & ~(GRAN - 1); }

// First-fit allocator of byte offsets in [0, size); free ranges coalesce.
class Arena {
  public:
    void init(size_t size) {
        size_ = size & ~(GRAN - 1);
        free_.clear();
        if (size_) free_[0] = size_;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = al(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t o = it->first, rem = it->second - bytes;
            free_.erase(it);
            if (rem) free_[o + bytes] = rem;
            used_ += bytes;
            *off = o;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = al(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

int elem_bytes(int dt) { return dt == MXP_F64 ? 8 : dt == MXP_F32 ? 4 : dt == MXP_F8E4M3 ? 1 : 2; }

// Device layout of one request inside its arena block.
struct ReqLayout {
    int64_t lda;
    size_t A, B, X, diag, ainf, aux, fwork, swork;
    size_t fwork_bytes, swork_bytes, total;
};

ReqLayout req_layout(int64_t n, int64_t nrhs, int64_t nb, int update, int store, int restart) {
    ReqLayout L;
    L.lda = (n + 63) / 64 * 64;   // 16-bit columns start on 128-byte boundaries
    size_t off = 0;
    L.A = off; off = al(off + (size_t)L.lda * n * elem_bytes(store));
    L.B = off; off = al(off + (size_t)n * nrhs * 8);
    L.X = off; off = al(off + (size_t)n * nrhs * 8);
    L.diag = off; off = al(off + (size_t)n * 8);
    L.ainf = off; off = al(off + 8);
    L.aux = off; off = al(off + mxp_factor_aux_bytes(n, nb));
    L.fwork_bytes = mxp_factor_work_bytes(n, nb, update);
    L.fwork = off; off = al(off + L.fwork_bytes);
    L.swork_bytes = mxp_solve_work_bytes(n, nrhs, restart);
    L.swork = off; off = al(off + L.swork_bytes);
    L.total = off;
    return L;
}

struct Req {
    uint64_t id = 0;
    int64_t n = 0, nrhs = 0, nb = 0;
    uint64_t seed = 0;
    double* x_host = nullptr;
    size_t bytes = 0, off = 0;
    int status = MXP_OK;
    int64_t iters = 0;
    double eta = 0;
    int64_t t_submit = 0, t_start = 0, t_done = 0;
    bool done = false;
};

constexpr int NCLASS = 6;           // size classes 512 << c
const int64_t NB_CANDIDATES[] = {128, 256, 512};
const int TILE_CANDIDATES[] = {MXP_TILE_256x128, MXP_TILE_128x128};
constexpr int MAX_WORKERS = 3;
constexpr int MAX_GROUP = 8;

int size_class(int64_t n) {
    const int c = (int)std::lround(std::log2((double)std::max<int64_t>(n, 1))) - 9;
    return std::min(std::max(c, 0), NCLASS - 1);
}

}  // namespace
}  // namespace mxp

using namespace mxp;

struct mxp_server {
    int device = 0;
    char* base = nullptr;
    mxp_server_cfg cfg{};
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    struct Worker {
        std::thread th;
        hipStream_t s = nullptr;
    };
    std::vector<Worker> workers;
    int group_max = 1;
    int64_t submitted = 0, completed = 0, failed = 0, in_flight = 0, peak_in_flight = 0, groups = 0,
            grouped_requests = 0, peak_group = 0;
    size_t peak_bytes = 0;
    int64_t nb_class[NCLASS] = {128, 128, 256, 256, 512, 512};
    int tile_class[NCLASS] = {MXP_TILE_128x128, MXP_TILE_128x128, MXP_TILE_128x128,
                              MXP_TILE_256x128, MXP_TILE_256x128, MXP_TILE_256x128};
    std::chrono::steady_clock::time_point t0;

    int64_t now_ns() const {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
    }
    int64_t block_size(int64_t n) const { return cfg.nb > 0 ? cfg.nb : nb_class[size_class(n)]; }
    int tile(int64_t n) const { return tile_class[size_class(n)]; }
};

namespace {

struct ReqBufs {
    ReqLayout L;
    char* b;
    void* A;
    double *B, *X, *diag, *ainf;
};

ReqBufs bufs_of(mxp_server* S, Req* r) {
    const mxp_server_cfg& c = S->cfg;
    ReqBufs q;
    q.L = req_layout(r->n, r->nrhs, r->nb, c.update, c.store, c.restart);
    q.b = S->base + r->off;
    q.A = q.b + q.L.A;
    q.B = (double*)(q.b + q.L.B);
    q.X = (double*)(q.b + q.L.X);
    q.diag = (double*)(q.b + q.L.diag);
    q.ainf = (double*)(q.b + q.L.ainf);
    return q;
}

// generate + factor (grouped) + refine a group of requests in their arena
// blocks on the worker's stream; each request is completed as soon as its
// own refinement is done
void run_group(mxp_server* S, mxp_server::Worker& w, std::vector<Req*>& grp, bool dev_ok) {
    const mxp_server_cfg& c = S->cfg;
    const int G = (int)grp.size();
    std::vector<ReqBufs> bq((size_t)G);
    std::vector<int> rc((size_t)G, dev_ok ? MXP_OK : MXP_EHIP);
    std::vector<mxp_factor_item> items;
    std::vector<int> idx;
    for (int g = 0; g < G && dev_ok; ++g) {
        Req* r = grp[(size_t)g];
        bq[(size_t)g] = bufs_of(S, r);
        const ReqBufs& q = bq[(size_t)g];
        rc[(size_t)g] = mxp_generate(r->n, r->nrhs, r->seed, MXP_GEN_DOMINANT, 0.0, c.store, q.A, q.L.lda, q.B, r->n,
                                     q.diag, nullptr, q.ainf, w.s);
        if (rc[(size_t)g]) continue;
        items.push_back(mxp_factor_item{r->n, r->nb, q.A, q.L.lda, q.b + q.L.aux, q.b + q.L.fwork, q.L.fwork_bytes});
        idx.push_back(g);
    }
    if (!items.empty()) {
        std::vector<int64_t> info(items.size(), 0);
        const int frc = mxp_factor_group((int)items.size(), items.data(), c.update, c.store, S->tile(grp[(size_t)idx[0]]->n),
                                         info.data(), w.s);
        for (size_t i = 0; i < idx.size(); ++i)
            if (frc < 0 || info[i]) rc[(size_t)idx[i]] = frc < 0 ? frc : MXP_ESINGULAR;
    }
    for (int g = 0; g < G; ++g) {
        Req* r = grp[(size_t)g];
        if (rc[(size_t)g] == MXP_OK) {
            const ReqBufs& q = bq[(size_t)g];
            std::vector<mxp_rhs_report> rep((size_t)r->nrhs);
            int s = mxp_solve_ir(r->n, r->nb, c.update, c.store, r->seed, MXP_GEN_DOMINANT, q.A, q.L.lda,
                                 q.b + q.L.aux, q.diag, q.ainf, q.B, r->n, q.X, r->n, r->nrhs, c.restart, c.max_iters,
                                 c.tol, c.tau, rep.data(), q.b + q.L.swork, q.L.swork_bytes, w.s);
            for (const mxp_rhs_report& x : rep) {
                r->iters = std::max<int64_t>(r->iters, x.iters);
                r->eta = std::max(r->eta, x.eta);
            }
            if (s >= 0 && r->x_host &&
                (hipMemcpyAsync(r->x_host, q.X, (size_t)r->n * r->nrhs * 8, hipMemcpyDeviceToHost, w.s) != hipSuccess ||
                 hipStreamSynchronize(w.s) != hipSuccess))
                s = MXP_EHIP;
            rc[(size_t)g] = s;
        }
        {
            std::lock_guard<std::mutex> lock(S->mu);
            S->arena.release(r->off, r->bytes);
            r->status = rc[(size_t)g];
            r->t_done = S->now_ns();
            r->done = true;
            S->in_flight--;
            if (r->status == MXP_OK) S->completed++;
            else S->failed++;
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
}

void worker_main(mxp_server* S, int k) {
    mxp_server::Worker& w = S->workers[(size_t)k];
    // a worker that cannot select the server's device fails every request it takes
    const bool dev_ok = hipSetDevice(S->device) == hipSuccess;
    for (;;) {
        std::vector<Req*> grp;
        {
            std::unique_lock<std::mutex> lock(S->mu);
            // the queue's head requests, in arrival order, while a slot is
            // free and their bytes fit in the arena
            S->cv_work.wait(lock, [&] {
                if (S->stop) return true;
                while (!S->queue.empty() && (int)grp.size() < S->group_max && S->in_flight < S->cfg.max_slots) {
                    size_t off;
                    Req* r = S->queue.front();
                    if (!S->arena.alloc(r->bytes, &off)) break;
                    r->off = off;
                    r->t_start = S->now_ns();
                    S->queue.pop_front();
                    S->in_flight++;
                    grp.push_back(r);
                }
                return !grp.empty();
            });
            if (S->stop && grp.empty()) return;   // destroy drains first: nothing is queued any more
            S->peak_in_flight = std::max(S->peak_in_flight, S->in_flight);
            S->peak_bytes = std::max(S->peak_bytes, S->arena.used());
            S->groups++;
            S->grouped_requests += (int64_t)grp.size();
            S->peak_group = std::max<int64_t>(S->peak_group, (int64_t)grp.size());
        }
        run_group(S, w, grp, dev_ok);
    }
}

// time factor + refinement of one size class for every candidate pair of
// block size and trailing-update tile
void autotune(mxp_server* S) {
    mxp_server::Worker& w = S->workers[0];
    const mxp_server_cfg& c = S->cfg;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return;
    }
    for (int cls = 0; cls < NCLASS; ++cls) {
        const int64_t n = 512ll << cls;
        float best = 0;
        for (int64_t nb : NB_CANDIDATES) {
            if (c.update == MXP_F8E4M3 && nb % 128) continue;
            const ReqLayout L = req_layout(n, 1, nb, c.update, c.store, c.restart);
            if (L.total > S->arena.size()) continue;
            for (int tile : TILE_CANDIDATES) {
                float ms_min = 0;
                bool ok = true;
                for (int rep = 0; rep < 3 && ok; ++rep) {
                    // regenerated each time (the factorisation overwrites A); generation is not timed
                    char* b = S->base;
                    if (mxp_generate(n, 1, 12345, MXP_GEN_DOMINANT, 0.0, c.store, b + L.A, L.lda, (double*)(b + L.B),
                                     n, (double*)(b + L.diag), nullptr, (double*)(b + L.ainf), w.s)) {
                        ok = false;
                        break;
                    }
                    if (hipEventRecord(e0, w.s) != hipSuccess) { ok = false; break; }
                    int64_t info = 0;
                    mxp_factor_item it{n, nb, b + L.A, L.lda, b + L.aux, b + L.fwork, L.fwork_bytes};
                    std::vector<mxp_rhs_report> q(1);
                    int rc = mxp_factor_group(1, &it, c.update, c.store, tile, &info, w.s);
                    if (!rc)
                        rc = mxp_solve_ir(n, nb, c.update, c.store, 12345, MXP_GEN_DOMINANT, b + L.A, L.lda, b + L.aux,
                                          (double*)(b + L.diag), (double*)(b + L.ainf), (double*)(b + L.B), n,
                                          (double*)(b + L.X), n, 1, c.restart, c.max_iters, c.tol, c.tau, q.data(),
                                          b + L.swork, L.swork_bytes, w.s);
                    if (rc != MXP_OK || hipEventRecord(e1, w.s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        ok = false;
                        break;
                    }
                    float ms = 0;
                    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { ok = false; break; }
                    if (rep > 0 && (ms_min == 0 || ms < ms_min)) ms_min = ms;   // the first run warms up
                }
                if (ok && (best == 0 || ms_min < best)) {
                    best = ms_min;
                    S->nb_class[cls] = nb;
                    S->tile_class[cls] = tile;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace

extern "C" size_t mxp_server_request_bytes(int64_t n, int64_t nrhs, int64_t nb, int update, int store, int restart) {
    if (n < 1 || nrhs < 1 || nb < 64 || restart < 1 || restart > 64) return 0;
    return req_layout(n, nrhs, nb, update, store, restart).total;
}

extern "C" int mxp_server_create(int device, void* arena, size_t arena_bytes, const mxp_server_cfg* cfg,
                                 mxp_server** out) {
    if (!arena || !cfg || !out || cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->restart < 1 ||
        cfg->restart > 64 || cfg->max_iters < 1 || !(cfg->tol > 0) || !(cfg->tau >= 0) ||
        (cfg->nb != 0 && (cfg->nb % 64 || cfg->nb > 1024)))
        return MXP_EINVAL;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return MXP_EHIP;
    std::unique_ptr<mxp_server> S(new mxp_server());
    S->device = device;
    S->base = (char*)arena;
    S->cfg = *cfg;
    S->arena.init(arena_bytes);
    S->t0 = std::chrono::steady_clock::now();
    // a few workers with one stream each, groups that share the slots
    const int nw = std::min(cfg->max_slots, MAX_WORKERS);
    S->group_max = std::min(MAX_GROUP, (cfg->max_slots + nw - 1) / nw);
    S->workers.resize((size_t)nw);
    int rc = MXP_OK;
    for (auto& w : S->workers) {
        if (hipStreamCreateWithFlags(&w.s, hipStreamNonBlocking) != hipSuccess) {
            rc = MXP_EHIP;
            break;
        }
    }
    if (rc == MXP_OK && cfg->autotune && cfg->nb == 0) autotune(S.get());
    if (rc != MXP_OK) {
        for (auto& w : S->workers)
            if (w.s) (void)hipStreamDestroy(w.s);
        (void)hipSetDevice(prev);   // restores the caller's device
        return rc;
    }
    for (int k = 0; k < nw; ++k) S->workers[(size_t)k].th = std::thread(worker_main, S.get(), k);
    (void)hipSetDevice(prev);
    *out = S.release();
    return MXP_OK;
}

extern "C" int mxp_server_submit(mxp_server* S, int64_t n, int64_t nrhs, uint64_t seed, double* x_host,
                                 uint64_t* id) {
    if (!S || !id || n < 1 || n >= (1ll << 31) || nrhs < 1 || nrhs > 64) return MXP_EINVAL;
    std::unique_ptr<Req> r(new Req());
    r->n = n;
    r->nrhs = nrhs;
    r->seed = seed;
    r->x_host = x_host;
    r->nb = S->block_size(n);
    r->bytes = req_layout(n, nrhs, r->nb, S->cfg.update, S->cfg.store, S->cfg.restart).total;
    if (r->bytes > S->arena.size()) return MXP_EINVAL;   // could never be admitted
    {
        std::lock_guard<std::mutex> lock(S->mu);
        r->id = S->next_id++;
        r->t_submit = S->now_ns();
        *id = r->id;
        S->queue.push_back(r.get());
        S->reqs.emplace(r->id, std::move(r));
        S->submitted++;
    }
    S->cv_work.notify_all();
    return MXP_OK;
}

static void fill_result(const Req& r, mxp_request_result* out) {
    out->id = r.id;
    out->n = r.n;
    out->nrhs = r.nrhs;
    out->nb = r.nb;
    out->status = r.status;
    out->pad = 0;
    out->iters = r.iters;
    out->eta = r.eta;
    out->t_submit_ns = r.t_submit;
    out->t_start_ns = r.t_start;
    out->t_done_ns = r.t_done;
}

extern "C" int mxp_server_poll(mxp_server* S, uint64_t id, mxp_request_result* out) {
    if (!S || !out) return MXP_EINVAL;
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return MXP_EINVAL;
    if (!it->second->done) return MXP_PENDING;
    fill_result(*it->second, out);
    return MXP_OK;
}

extern "C" int mxp_server_wait(mxp_server* S, uint64_t id, mxp_request_result* out) {
    if (!S || !out) return MXP_EINVAL;
    std::unique_lock<std::mutex> lock(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return MXP_EINVAL;
    Req* r = it->second.get();
    S->cv_done.wait(lock, [&] { return r->done; });
    fill_result(*r, out);
    return MXP_OK;
}

extern "C" int mxp_server_drain(mxp_server* S) {
    if (!S) return MXP_EINVAL;
    std::unique_lock<std::mutex> lock(S->mu);
    S->cv_done.wait(lock, [&] { return S->completed + S->failed == S->submitted; });
    return MXP_OK;
}

extern "C" int mxp_server_get_stats(mxp_server* S, mxp_server_stats* out) {
    if (!S || !out) return MXP_EINVAL;
    std::lock_guard<std::mutex> lock(S->mu);
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->failed = S->failed;
    out->in_flight = S->in_flight;
    out->peak_in_flight = S->peak_in_flight;
    out->arena_bytes = S->arena.size();
    out->bytes_in_use = S->arena.used();
    out->peak_bytes_in_use = S->peak_bytes;
    out->groups = S->groups;
    out->grouped_requests = S->grouped_requests;
    out->peak_group = S->peak_group;
    out->streams = (int64_t)S->workers.size();
    return MXP_OK;
}

extern "C" int64_t mxp_server_block_size(mxp_server* S, int64_t n) { return S ? S->block_size(n) : 0; }

extern "C" int mxp_server_tile(mxp_server* S, int64_t n) { return S ? S->tile(n) : -1; }

extern "C" int mxp_server_destroy(mxp_server* S) {
    if (!S) return MXP_EINVAL;
    mxp_server_drain(S);
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& w : S->workers)
        if (w.th.joinable()) w.th.join();
    // teardown: the streams are released on the server's device, whatever
    // those calls return
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    for (auto& w : S->workers)
        if (w.s) (void)hipStreamDestroy(w.s);
    (void)hipSetDevice(prev);
    delete S;
    return MXP_OK;
}
