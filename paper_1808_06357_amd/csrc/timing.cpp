// Per-kernel-class HIP-event timing of the launches the library makes.  When
// enabled, every launch gets a start / stop event pair that the kernel
// dispatch itself stamps (hipExtLaunchKernelGGL), so the elapsed time is the
// kernel's own duration without extra marker packets in the stream;
// lt_timing_summary waits for them and sums the elapsed times.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "lt_internal.h"

namespace lt {
namespace {
struct Rec {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take()
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

void timing_events(int kind, void **start, void **stop)
{
    *start = *stop = nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    hipEvent_t a = take(), b = take();
    if (!a || !b) return;
    g_recs.push_back({kind, a, b});
    *start = a;
    *stop = b;
}

}  // namespace lt

extern "C" lt_status lt_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(lt::g_mu);
    for (auto &r : lt::g_recs) {
        hipEventSynchronize(r.b);
        lt::g_pool.push_back(r.a);
        lt::g_pool.push_back(r.b);
    }
    lt::g_recs.clear();
    lt::g_on = on != 0;
    return LT_OK;
}

extern "C" lt_status lt_timing_summary(int32_t kind, int64_t *launches, double *total_ms)
{
    if (!launches || !total_ms) return lt::fail(LT_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(lt::g_mu);
    int64_t n = 0;
    double ms = 0.0;
    for (auto &r : lt::g_recs) {
        if (r.kind != kind) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return lt::fail(LT_E_HIP, "event wait failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return lt::fail(LT_E_HIP, "event time failed");
        ms += t;
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    return LT_OK;
}
