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
//   * slots: each is a host thread with its own stream and look-ahead
//     context, so the kernels of requests in flight overlap on the device;
//   * a block-size tuner: per size class (powers of two 512 .. 16384) the
//     candidate block sizes are timed on the device at creation and the
//     fastest is kept.
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
    struct Slot {
        std::thread th;
        hipStream_t s = nullptr;
        Lookahead la;
    };
    std::vector<Slot> slots;
    int64_t submitted = 0, completed = 0, failed = 0, in_flight = 0, peak_in_flight = 0;
    size_t peak_bytes = 0;
    int64_t nb_class[NCLASS] = {128, 128, 256, 256, 512, 512};
    std::chrono::steady_clock::time_point t0;

    int64_t now_ns() const {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
    }
    int64_t block_size(int64_t n) const { return cfg.nb > 0 ? cfg.nb : nb_class[size_class(n)]; }
};

namespace {

// generate + factor + refine one request in its arena block, on the slot's
// stream; returns the first non-OK status
int run_request(mxp_server* S, mxp_server::Slot& sl, Req* r) {
    const mxp_server_cfg& c = S->cfg;
    const ReqLayout L = req_layout(r->n, r->nrhs, r->nb, c.update, c.store, c.restart);
    char* b = S->base + r->off;
    void* A = b + L.A;
    double* B = (double*)(b + L.B);
    double* X = (double*)(b + L.X);
    double* diag = (double*)(b + L.diag);
    double* ainf = (double*)(b + L.ainf);
    int rc = mxp_generate(r->n, r->nrhs, r->seed, c.store, A, L.lda, B, r->n, diag, ainf, sl.s);
    if (rc) return rc;
    int64_t info = 0;
    rc = factor_with(r->n, r->nb, c.update, c.store, MXP_SCALE_NONE, diag, A, L.lda, b + L.aux, b + L.fwork,
                     L.fwork_bytes, &info, sl.s, &sl.la);
    if (rc) return rc;
    std::vector<mxp_rhs_report> rep((size_t)r->nrhs);
    rc = mxp_solve_ir(r->n, r->nb, c.update, c.store, r->seed, A, L.lda, b + L.aux, diag, ainf, B, r->n, X, r->n,
                      r->nrhs, c.restart, c.max_iters, c.tol, c.tau, rep.data(), b + L.swork, L.swork_bytes, sl.s);
    for (const mxp_rhs_report& q : rep) {
        r->iters = std::max<int64_t>(r->iters, q.iters);
        r->eta = std::max(r->eta, q.eta);
    }
    if (rc < 0) return rc;
    if (r->x_host) {
        if (hipMemcpyAsync(r->x_host, X, (size_t)r->n * r->nrhs * 8, hipMemcpyDeviceToHost, sl.s) != hipSuccess ||
            hipStreamSynchronize(sl.s) != hipSuccess)
            return MXP_EHIP;
    }
    return rc;
}

void slot_main(mxp_server* S, int k) {
    mxp_server::Slot& sl = S->slots[(size_t)k];
    // a slot that cannot select the server's device fails every request it takes
    const bool dev_ok = hipSetDevice(S->device) == hipSuccess;
    for (;;) {
        Req* r = nullptr;
        {
            std::unique_lock<std::mutex> lock(S->mu);
            S->cv_work.wait(lock, [&] {
                if (S->stop) return true;
                size_t off;
                if (S->queue.empty() || !S->arena.alloc(S->queue.front()->bytes, &off)) return false;
                S->queue.front()->off = off;
                return true;
            });
            if (S->stop) return;   // destroy drains first: nothing is queued any more
            r = S->queue.front();
            S->queue.pop_front();
            r->t_start = S->now_ns();
            S->in_flight++;
            S->peak_in_flight = std::max(S->peak_in_flight, S->in_flight);
            S->peak_bytes = std::max(S->peak_bytes, S->arena.used());
        }
        const int rc = dev_ok ? run_request(S, sl, r) : MXP_EHIP;
        {
            std::lock_guard<std::mutex> lock(S->mu);
            S->arena.release(r->off, r->bytes);
            r->status = rc;
            r->t_done = S->now_ns();
            r->done = true;
            S->in_flight--;
            if (rc == MXP_OK) S->completed++;
            else S->failed++;
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
}

// time factor + refinement of one size class for every candidate block size
void autotune(mxp_server* S) {
    mxp_server::Slot& sl = S->slots[0];
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
            const ReqLayout L = req_layout(n, 1, nb, c.update, c.store, c.restart);
            if (L.total > S->arena.size()) continue;
            Req r;
            r.n = n; r.nrhs = 1; r.nb = nb; r.seed = 12345; r.off = 0;
            float ms_min = 0;
            bool ok = true;
            for (int rep = 0; rep < 3 && ok; ++rep) {
                // regenerated each time (the factorisation overwrites A); generation is not timed
                char* b = S->base;
                if (mxp_generate(n, 1, r.seed, c.store, b + L.A, L.lda, (double*)(b + L.B), n, (double*)(b + L.diag),
                                 (double*)(b + L.ainf), sl.s)) { ok = false; break; }
                if (hipEventRecord(e0, sl.s) != hipSuccess) { ok = false; break; }
                int64_t info = 0;
                std::vector<mxp_rhs_report> q(1);
                int rc = factor_with(n, nb, c.update, c.store, MXP_SCALE_NONE, (double*)(b + L.diag), b + L.A, L.lda,
                                     b + L.aux, b + L.fwork, L.fwork_bytes, &info, sl.s, &sl.la);
                if (!rc)
                    rc = mxp_solve_ir(n, nb, c.update, c.store, r.seed, b + L.A, L.lda, b + L.aux,
                                      (double*)(b + L.diag), (double*)(b + L.ainf), (double*)(b + L.B), n,
                                      (double*)(b + L.X), n, 1, c.restart, c.max_iters, c.tol, c.tau, q.data(),
                                      b + L.swork, L.swork_bytes, sl.s);
                if (rc != MXP_OK || hipEventRecord(e1, sl.s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
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
    S->slots.resize((size_t)cfg->max_slots);
    int rc = MXP_OK;
    for (auto& sl : S->slots) {
        if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess || lookahead_create(&sl.la)) {
            rc = MXP_EHIP;
            break;
        }
    }
    if (rc == MXP_OK && cfg->autotune && cfg->nb == 0) autotune(S.get());
    if (rc != MXP_OK) {
        for (auto& sl : S->slots) {
            lookahead_destroy(&sl.la);
            if (sl.s) (void)hipStreamDestroy(sl.s);
        }
        (void)hipSetDevice(prev);   // restores the caller's device
        return rc;
    }
    for (int k = 0; k < cfg->max_slots; ++k) S->slots[(size_t)k].th = std::thread(slot_main, S.get(), k);
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
    return MXP_OK;
}

extern "C" int64_t mxp_server_block_size(mxp_server* S, int64_t n) { return S ? S->block_size(n) : 0; }

extern "C" int mxp_server_destroy(mxp_server* S) {
    if (!S) return MXP_EINVAL;
    mxp_server_drain(S);
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& sl : S->slots)
        if (sl.th.joinable()) sl.th.join();
    // teardown: the streams and events are released on the server's device,
    // whatever those calls return
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    for (auto& sl : S->slots) {
        lookahead_destroy(&sl.la);
        if (sl.s) (void)hipStreamDestroy(sl.s);
    }
    (void)hipSetDevice(prev);
    delete S;
    return MXP_OK;
}
