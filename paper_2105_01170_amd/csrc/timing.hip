// Per-kernel timing for diagnostics and for measuring the roofline of a single
// kernel inside a multi-kernel call.  While enabled, every launch the library
// makes is bracketed by two HIP events recorded on the launch stream; the
// records are reduced per kernel name on request.  Disabled (the default),
// the launch path only tests one flag.
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace tsvdm {

bool g_trace = false;

namespace {
struct Rec {
    const char *name;
    hipEvent_t a, b;
};
struct Agg {
    std::string name;
    int launches;
    double ms;
};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<Agg> g_aggs;
hipEvent_t g_pending = nullptr;
const char *g_pending_name = nullptr;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

void trace_begin(const char *name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending = get_event();
    g_pending_name = name;
    if (g_pending && hipEventRecord(g_pending, s) != hipSuccess) {  // the launch goes untimed
        g_pool.push_back(g_pending);
        g_pending = nullptr;
    }
}

void trace_end(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_pending) return;
    hipEvent_t b = get_event();
    if (!b) return;
    if (hipEventRecord(b, s) == hipSuccess) {
        g_recs.push_back({g_pending_name, g_pending, b});
    } else {  // the launch goes untimed
        g_pool.push_back(b);
        g_pool.push_back(g_pending);
    }
    g_pending = nullptr;
}

}  // namespace tsvdm

using namespace tsvdm;

extern "C" {

tsvdm_status tsvdm_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_trace = on != 0;
    if (g_trace) {  // a fresh window
        for (auto &r : g_recs) {
            g_pool.push_back(r.a);
            g_pool.push_back(r.b);
        }
        g_recs.clear();
        g_aggs.clear();
    }
    return TSVDM_OK;
}

int32_t tsvdm_timing_count(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_aggs.clear();
    for (auto &r : g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
        Agg *hit = nullptr;
        for (auto &g : g_aggs)
            if (g.name == r.name) hit = &g;
        if (!hit) {
            g_aggs.push_back({r.name, 0, 0.0});
            hit = &g_aggs.back();
        }
        hit->launches += 1;
        hit->ms += ms;
    }
    return (int32_t)g_aggs.size();
}

tsvdm_status tsvdm_timing_get(int32_t i, const char **name, int32_t *launches, double *total_ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int32_t)g_aggs.size() || !name || !launches || !total_ms) {
        set_error("tsvdm_timing_get: index %d out of range or NULL output", i);
        return TSVDM_EINVAL;
    }
    *name = g_aggs[i].name.c_str();
    *launches = g_aggs[i].launches;
    *total_ms = g_aggs[i].ms;
    return TSVDM_OK;
}

}  // extern "C"
