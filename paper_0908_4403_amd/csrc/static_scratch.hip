// Library-owned device workspace of fixed size for heget_xsec_device_noalloc,
// the cross-section entry point for callers that cannot allocate (graph
// capture, serving loops).  The array lives in the code object; each device
// that loads the library holds its own copy until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current and kept here; only that address is ever handed to
// kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace heget {

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

// Device address of the workspace on the current device (looked up on the
// first call per device).
hipError_t static_scratch_ptr(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_static_ptr[dev] = p;
    }
    *ptr = g_static_ptr[dev];
    return hipSuccess;
}

}  // namespace heget
