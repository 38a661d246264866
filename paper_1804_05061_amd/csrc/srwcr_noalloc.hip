// srwcr_noalloc.hip -- srwcr_grad for callers that cannot allocate device
// memory: the workspace is a static device array of this library, one per
// device, instead of a caller's buffer (see include/srwcr.h).
#include <hip/hip_runtime.h>

#include <mutex>

#include "srwcr.h"
#include "srwcr_internal.h"

using namespace srwcr;

namespace {

constexpr size_t kScratchBytes = (size_t)SRWCR_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The workspace of srwcr_grad_noalloc.  In host code `scratch` names a host
// stand-in, not device memory: kernels get the address hipGetSymbolAddress
// returns for the current device, never the array's name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The current device's copy of `scratch`, looked up once per device.
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return report_error(SRWCR_E_UNSUPPORTED, "device %d is beyond the %d the static workspace tracks", dev,
                            kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return report_error(SRWCR_E_HIP, "hipGetSymbolAddress(static workspace) on device %d: %s", dev,
                                hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SRWCR_OK;
}

}  // namespace

extern "C" int srwcr_grad_noalloc(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd,
                                  double *d_value, float *d_grad, void *stream)
{
    if (!plan) return report_error(SRWCR_E_INVALID_ARG, "plan is NULL");
    const size_t need = srwcr_workspace_bytes(plan);
    if (need > kScratchBytes)
        return report_error(SRWCR_E_WORKSPACE,
                            "the plan needs %zu B of workspace; the static workspace of srwcr_grad_noalloc holds %zu B",
                            need, kScratchBytes);
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report_error(SRWCR_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev != plan_device(plan))
        return report_error(SRWCR_E_INVALID_ARG, "the current device %d is not the plan's device %d", dev,
                            plan_device(plan));
    void *ws = nullptr;
    const int st = scratch_address(dev, &ws);
    if (st) return st;
    return srwcr_grad(plan, fixed, moving, ffd, d_value, d_grad, ws, kScratchBytes, stream);
}
