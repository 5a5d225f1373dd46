// prof.hip -- event pool and accumulation behind prof.hpp and the
// mxp_profile_* entry points.
#include <mutex>
#include <vector>

#include "../../include/mxp.h"
#include "prof.hpp"

namespace mxp {
namespace prof {

struct Rec {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
};

static std::mutex g_mu;
static int g_mask = 0;                   // bit c: class c is timed
static std::vector<hipEvent_t> g_pool;   // free events
static std::vector<Rec> g_pending;       // recorded, not yet collected
static double g_ms[NCLS], g_flops[NCLS], g_bytes[NCLS];
static int64_t g_count[NCLS];

static hipEvent_t take() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool enabled() { return g_mask != 0; }

hipEvent_t begin(Cls c, hipStream_t s) {
    if (!(g_mask >> (int)c & 1)) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t a = take();
    // a record that fails leaves the launch untimed
    if (a && hipEventRecord(a, s) != hipSuccess) {
        g_pool.push_back(a);
        return nullptr;
    }
    return a;
}

void end(hipEvent_t a, Cls c, hipStream_t s, double flops, double bytes) {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take();
    if (!b || hipEventRecord(b, s) != hipSuccess) {
        g_pool.push_back(a);
        if (b) g_pool.push_back(b);
        return;
    }
    g_pending.push_back({(int)c, a, b, flops, bytes});
}

}  // namespace prof
}  // namespace mxp

using namespace mxp::prof;

extern "C" int mxp_profile_enable(int mask) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_mask = mask & ((1 << NCLS) - 1);
    return MXP_OK;
}

extern "C" int mxp_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_pending) { g_pool.push_back(r.a); g_pool.push_back(r.b); }
    g_pending.clear();
    for (int c = 0; c < NCLS; ++c) { g_ms[c] = g_flops[c] = g_bytes[c] = 0; g_count[c] = 0; }
    return MXP_OK;
}

extern "C" int mxp_profile_read(int cls, double* total_ms, double* flops, double* bytes, int64_t* launches) {
    if (cls < 0 || cls >= NCLS || !total_ms || !flops || !bytes || !launches) return MXP_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            return MXP_EHIP;
        g_ms[r.cls] += ms;
        g_flops[r.cls] += r.flops;
        g_bytes[r.cls] += r.bytes;
        g_count[r.cls] += 1;
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_pending.clear();
    *total_ms = g_ms[cls];
    *flops = g_flops[cls];
    *bytes = g_bytes[cls];
    *launches = g_count[cls];
    return MXP_OK;
}
