// Fixed device scratch of the no-allocation sampling entry point
// (tkdv_sample_noalloc): one statically sized array per GPU, holding the
// launch sequence's work buffers (accept bitmap, FP64 re-decision list,
// counters, segment arrays, point records).  The host never names the array
// itself: at context creation its device address is looked up once per device
// with that device current and kept; every later use goes through that
// address.  All calls on one GPU share the array, so calls that overlap on
// one GPU race.
#include <hip/hip_runtime.h>

#include "tkdv_scratch.h"

namespace tkdv {

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = ptr;
    if (cur != device) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    return e;
}

void *scratch_ptr(int device)
{
    return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace tkdv
