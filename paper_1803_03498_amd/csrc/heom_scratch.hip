// Library-owned device scratch for the entry point that allocates nothing
// (heom_propagate_noalloc): a file-scope device array, one copy per GPU.
//
// In host code the array's name is only a host-side handle: its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and only that address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "heom_internal.h"

namespace heom {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_buffer(void** out, size_t* bytes) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

}  // namespace heom
