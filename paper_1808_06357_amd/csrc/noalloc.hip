// strang_run without allocation: the run's workspace is a static device
// array of this library (one per GPU, held until the process ends) instead of
// caller memory or a stream-ordered allocation.  For callers that cannot
// allocate (graph capture, serving loops, harnesses that forbid it).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lt_internal.h"

namespace {
// the largest workspace the entry point serves: a complex128 run of one
// state on the 2^20-point chirp-z lattice (transform buffer, convolution
// spectrum and scratch, merged potential table) needs 96 MiB
constexpr size_t kScratchBytes = size_t(128) << 20;
}  // namespace

// this GPU's run workspace; host code reaches its device address only
// through hipGetSymbolAddress (scratch_ptr)
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// the device address of this GPU's copy of the array (the name of the array
// in host code is a host-side stand-in, not a device address)
lt_status scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lt::fail(LT_E_HIP, std::string("device query: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return lt::fail(LT_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return lt::fail(LT_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LT_OK;
}

}  // namespace

extern "C" {

lt_status strang_run_noalloc_capacity(size_t *bytes)
{
    if (!bytes) return lt::fail(LT_E_ARG, "bytes is NULL");
    *bytes = kScratchBytes;
    return LT_OK;
}

lt_status strang_run_noalloc(const lt_plan *cp, lt_prec prec, int32_t batch, const double *v, int64_t v_stride,
                             void *u, double gamma, double dt, int64_t steps, void *stream)
{
    if (!cp) return lt::fail(LT_E_ARG, "plan is NULL");
    if (prec != LT_C64 && prec != LT_C128) return lt::fail(LT_E_ARG, "prec must be LT_C64 or LT_C128");
    if (batch < 0) return lt::fail(LT_E_ARG, "batch must be >= 0");
    lt_plan &p = *const_cast<lt_plan *>(cp);
    size_t need = 0;
    lt_status st = strang_workspace_size(cp, prec, batch, v_stride == 0, &need);
    if (st) return st;
    if (need > kScratchBytes)
        return lt::fail(LT_E_ARG, "strang_run_noalloc: the run needs " + std::to_string(need) +
                                      " bytes of workspace; its static scratch holds " +
                                      std::to_string(kScratchBytes));
    if (batch > 0 && steps > 0 && p.sched[0][prec].ok && !lt::forward_tables_ready(p, prec))
        return lt::fail(LT_E_ARG, "strang_run_noalloc: the plan's device tables for this precision are not "
                                  "built (create the plan with this precision in prec_mask, or run it once)");
    void *ws = nullptr;
    if ((st = scratch_ptr(&ws))) return st;
    return strang_run(cp, prec, batch, v, v_stride, u, gamma, dt, steps, nullptr, 0, ws, kScratchBytes, stream);
}

}  // extern "C"
