// Workspace-free variant of the batched evolution, for callers that cannot
// allocate device memory: its work lists go to a library-held device array
// instead of a caller buffer.

#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/tsq.h"
#include "tsq_internal.h"

namespace {

// Work lists of one tsq_batch_evolve_noalloc call.  Each GPU the library runs
// on holds its own copy until the process ends; every call on that GPU reuses
// it, so calls that overlap on one GPU race.
constexpr size_t kScratchBytes = tsq::kNoAllocScratchBytes;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of `scratch` per device (host-side name is not one)

// Address of this device's copy of `scratch`, looked up once per device with
// that device current.
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int tsq_batch_evolve_noalloc(tsq_plan* const* plans, void* const* psi_dev,
                                        void* const* ws, const int64_t* steps, int32_t n,
                                        const tsq_schedule* schedule, void* stream) {
    void* p = nullptr;
    const hipError_t e = scratch_address(&p);
    if (e != hipSuccess)
        return tsq::set_error(TSQ_ERR_DEVICE, "scratch address of tsq_batch_evolve_noalloc: %s",
                              hipGetErrorString(e));
    size_t need = 0;
    const int rc = tsq::batch_evolve_into(plans, psi_dev, ws, steps, n, schedule, p, kScratchBytes,
                                          stream, &need);
    if (rc == TSQ_ERR_WORKSPACE && need > kScratchBytes)
        return tsq::set_error(TSQ_ERR_WORKSPACE,
                              "the batch's work lists take %zu bytes, more than the %zu bytes "
                              "tsq_batch_evolve_noalloc holds; use tsq_batch_evolve with a "
                              "workspace",
                              need, kScratchBytes);
    return rc;
}
