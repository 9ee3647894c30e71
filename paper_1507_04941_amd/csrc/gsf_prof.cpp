// gsf_prof.cpp -- optional per-kernel timing with hipEvents (gsf_profile_*).
#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gsf_internal.h"

namespace {

struct Rec {
    const char *name;
    hipEvent_t start, stop;
};

struct Agg {
    const char *name;
    int64_t launches;
    double ms;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<Agg> g_agg;

hipEvent_t take_event()
{
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

namespace gsf {
namespace prof {

bool enabled() { return g_on.load(std::memory_order_relaxed); }

Scope::Scope(const char *name, hipStream_t s) : slot(-1), stream(s)
{
    if (!enabled()) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Rec r{name, take_event(), take_event()};
    if (!r.start || !r.stop) return;
    if (hipEventRecord(r.start, s) != hipSuccess) return;
    g_recs.push_back(r);
    slot = (int)g_recs.size() - 1;
}

Scope::~Scope()
{
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (slot < (int)g_recs.size()) (void)hipEventRecord(g_recs[slot].stop, stream);
}

}  // namespace prof
}  // namespace gsf

extern "C" {

gsf_status gsf_profile_enable(int on)
{
    g_on.store(on != 0);
    return GSF_OK;
}

gsf_status gsf_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (Rec &r : g_recs) {
        (void)hipEventSynchronize(r.stop);
        g_pool.push_back(r.start);
        g_pool.push_back(r.stop);
    }
    g_recs.clear();
    g_agg.clear();
    return GSF_OK;
}

int32_t gsf_profile_collect(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    std::map<std::string, Agg> m;
    for (const Rec &r : g_recs) {
        if (hipEventSynchronize(r.stop) != hipSuccess) return -1;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return -1;
        Agg &a = m[r.name];
        a.name = r.name;
        a.launches += 1;
        a.ms += ms;
    }
    g_agg.clear();
    for (auto &kv : m) g_agg.push_back(kv.second);
    return (int32_t)g_agg.size();
}

gsf_status gsf_profile_entry(int32_t i, const char **name, int64_t *launches, double *total_ms)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int32_t)g_agg.size() || !name || !launches || !total_ms)
        return GSF_ERR_INVALID_ARG;
    *name = g_agg[i].name;
    *launches = g_agg[i].launches;
    *total_ms = g_agg[i].ms;
    return GSF_OK;
}

}  // extern "C"
