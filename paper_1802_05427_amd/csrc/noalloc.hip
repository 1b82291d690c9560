// lmmse_estimate without a caller workspace, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The workspace is a file-scope device array of LMMSE_NOALLOC_SCRATCH_BYTES.
// Its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and cached; host code passes that address, never the
// array's name, to the kernels.  Each GPU holds its own copy of the array
// until the process ends, and every call on a GPU shares it: calls that
// overlap on one GPU (other streams, other threads) race.  Nothing in the
// estimate reads the workspace before writing it, so it is never cleared.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = LMMSE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of the array (the current device).
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return LMMSE_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LMMSE_ERR_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LMMSE_OK;
}

}  // namespace

extern "C" int lmmse_estimate_noalloc(lmmse_plan_t plan, int slots, const void* y_pilot,
                                      const void* pilots, double sigma2, void* h_hat,
                                      void* stream) {
    if (!plan) return LMMSE_ERR_INVALID_ARG;
    lmmse_plan_desc d;
    if (lmmse_plan_get_desc(plan, &d) != LMMSE_OK) return LMMSE_ERR_INVALID_ARG;
    if (slots < 0 || slots > d.max_slots) return LMMSE_ERR_INVALID_ARG;
    if (slots > 0 && lmmse::forward_workspace_bytes(d, slots) > kScratchBytes)
        return LMMSE_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LMMSE_ERR_HIP;
    if (dev != lmmse::plan_device(plan)) return LMMSE_ERR_INVALID_ARG;
    void* ws = nullptr;
    const int rc = scratch_address(dev, &ws);
    if (rc != LMMSE_OK) return rc;
    return lmmse_estimate(plan, slots, y_pilot, pilots, sigma2, h_hat, ws, kScratchBytes, stream);
}
