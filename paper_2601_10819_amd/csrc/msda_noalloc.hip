// msda_forward_noalloc: the forward for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc). The workspace msda_forward_ws takes from its caller -- the
// view-order forward's per-XCD-slot partial sums, and the softmax statistics
// when the weights are logits -- lives here in a fixed device array of
// MSDA_NOALLOC_SCRATCH_BYTES instead. Each GPU the library runs on holds its
// own copy of the array until the process ends; every call on that GPU uses
// it, so calls that overlap on one GPU (two streams, two threads) race.
// Nothing in it needs to start at zero: the forward overwrites every partial
// row it later reads (zeros for an anchor with no camera in a slot) and
// recomputes the statistics on every call.
#include <hip/hip_runtime.h>
#include <stdio.h>

#include <mutex>

#include "../../include/msda.h"
#include "msda_internal.h"

namespace {

constexpr size_t kScratchBytes = MSDA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The array itself. In host code its name is only a handle for
// hipGetSymbolAddress: kernels get the device address looked up below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per device: the array's device address, looked up once with that device
// current, and the lookup's status.
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_status[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];

msda_status failf(msda_status st, const char* fmt, size_t a, size_t b) {
    char buf[256];
    snprintf(buf, sizeof(buf), fmt, a, b);
    return msda::set_error(st, buf);
}

}  // namespace

extern "C" msda_status msda_forward_noalloc(const void* feat, const int32_t* spatial_shapes,
                                            const int32_t* level_start_index,
                                            const float* sampling_loc, const float* weights,
                                            float* out, const msda_desc* desc, void* stream) {
    if (!desc) return msda::set_error(MSDA_ERR_INVALID_ARGUMENT, "desc is NULL");
    // the size check comes first: no HIP call for an input that cannot fit
    const size_t need = msda_forward_workspace_size(desc);
    if (need > kScratchBytes)
        return failf(MSDA_ERR_UNSUPPORTED,
                     "msda_forward_noalloc: this input needs %zu bytes of scratch, more than the "
                     "fixed %zu (use msda_forward_ws with a workspace)",
                     need, kScratchBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return msda::set_error(MSDA_ERR_HIP, "msda_forward_noalloc: hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return failf(MSDA_ERR_UNSUPPORTED, "msda_forward_noalloc: device %zu (at most %zu)",
                     (size_t)dev, (size_t)kMaxDevices - 1);
    // once per device, with that device current (hipGetDevice just named it)
    std::call_once(g_scratch_once[dev], [dev]() {
        void* p = nullptr;
        g_scratch_status[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = p;
    });
    if (g_scratch_status[dev] != hipSuccess || !g_scratch_ptr[dev])
        return msda::set_error(MSDA_ERR_HIP,
                               "msda_forward_noalloc: hipGetSymbolAddress of the scratch array "
                               "failed");
    return msda_forward_ws(feat, spatial_shapes, level_start_index, sampling_loc, weights, out,
                           g_scratch_ptr[dev], kScratchBytes, desc, stream);
}
