// rt_noalloc.hip -- the device scratch array of the allocation-free backward
// (rt_lookup_bwd_noalloc): a file-scope array in device memory that takes the
// place of the caller's workspace, for callers that cannot allocate (code under
// HIP graph capture, serving loops that forbid allocation).
//
// Every GPU the library runs on holds its own copy of the array until the
// process ends.  In host code the array's name is a host-side stand-in, not a
// device address: the address is looked up once per device with
// hipGetSymbolAddress, that device current, and only that address is handed
// to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rt_device.hpp"
#include "rt_kernels.hpp"

namespace rt {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES];  // device address per device, nullptr until looked up
}  // namespace

hipError_t noalloc_scratch(void** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace rt
