// pm_equiprop_dev_noalloc: pm_equiprop_dev for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  The
// propagation kernel's only scratch memory -- the product tree's tickets and
// nodes -- lives in a fixed device array of this file instead of the
// context's workspace buffers.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pm_internal.h"

namespace {

// Tree workspace shared by every call on a device: tickets, then nodes.  A
// propagation whose tree needs more is refused (PM_E_INVALID_ARG).
constexpr size_t kScratchBytes = size_t(64) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` per device, taken once with that device current.
struct ScratchSlot {
    std::once_flag once;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};
ScratchSlot g_slots[kMaxDevices];

hipError_t scratch_address(int device, void** out) {
    ScratchSlot& s = g_slots[device];
    std::call_once(s.once, [&] {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        s.err = hipSetDevice(device);
        if (s.err == hipSuccess) s.err = hipGetSymbolAddress(&s.ptr, HIP_SYMBOL(scratch));
        if (s.err != hipSuccess) s.ptr = nullptr;
        if (prev >= 0) (void)hipSetDevice(prev);
    });
    *out = s.ptr;
    return s.err;
}

}  // namespace

extern "C" pm_status pm_equiprop_dev_noalloc(pm_ctx* ctx, const double* samples_dev, int64_t n_samples,
                                             double dt, double* U_out_dev, void* slices_out_dev, void* stream) {
    if (!ctx) return PM_E_INVALID_ARG;
    const int dev = pm::context_device(ctx);
    if (dev < 0 || dev >= kMaxDevices) return PM_E_UNSUPPORTED;
    void* ws = nullptr;
    const hipError_t e = scratch_address(dev, &ws);
    if (e != hipSuccess || !ws)
        return pm::context_device_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                       "hipGetSymbolAddress(scratch)");
    return pm::equiprop_fixed_workspace(ctx, samples_dev, n_samples, dt, U_out_dev, slices_out_dev, stream, ws,
                                        kScratchBytes);
}
