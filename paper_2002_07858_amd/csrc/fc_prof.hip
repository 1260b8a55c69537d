// fc_prof.hip -- optional kernel timing for measurement tools.
//
// While enabled, each launch of a scan kernel is bracketed by two HIP events
// recorded on the stream the kernel is launched on (ProfScope in the
// launchers); fc_profile_read waits for a kernel's events and sums their
// elapsed times.  Disabled (the default), a ProfScope costs one atomic load.
#include <atomic>
#include <mutex>
#include <string.h>

#include "fc_internal.h"

namespace fcx {

namespace {

struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};

std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t pool_get()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drop_records()
{
    for (auto &r : g_prof_recs) {
        if (r.a) g_prof_pool.push_back(r.a);
        if (r.b) g_prof_pool.push_back(r.b);
    }
    g_prof_recs.clear();
}

}  // namespace

ProfScope::ProfScope(hipStream_t st, const char *name) : st_(st), slot_(-1)
{
    if (!g_prof_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r{name, pool_get(), pool_get()};
    if (!r.a || !r.b || hipEventRecord(r.a, st) != hipSuccess) {
        if (r.a) g_prof_pool.push_back(r.a);
        if (r.b) g_prof_pool.push_back(r.b);
        return;
    }
    slot_ = (int)g_prof_recs.size();
    g_prof_recs.push_back(r);
}

ProfScope::~ProfScope()
{
    if (slot_ < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (slot_ < (int)g_prof_recs.size() && hipEventRecord(g_prof_recs[slot_].b, st_) != hipSuccess)
        g_prof_recs[slot_].name = nullptr;  // never completed: not counted
}

}  // namespace fcx

extern "C" {

int fc_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(fcx::g_prof_mu);
    fcx::drop_records();
    fcx::g_prof_on.store(on ? 1 : 0);
    return FC_OK;
}

int fc_profile_read(const char *kernel, int64_t *launches, double *total_ms)
{
    if (!kernel || !launches || !total_ms)
        return fcx::set_last_error(FC_ERR_INVALID_ARG, "fc_profile_read: NULL argument");
    std::lock_guard<std::mutex> lk(fcx::g_prof_mu);
    int64_t n = 0;
    double ms = 0.0;
    for (auto &r : fcx::g_prof_recs) {
        if (!r.name || strcmp(r.name, kernel) != 0) continue;
        float t = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)
            return fcx::set_last_error(FC_ERR_DEVICE, "fc_profile_read: event query failed");
        ++n;
        ms += t;
    }
    *launches = n;
    *total_ms = ms;
    return FC_OK;
}

}  // extern "C"
