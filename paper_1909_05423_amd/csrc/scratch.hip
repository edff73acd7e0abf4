// The fixed device buffer behind pp_solve_noalloc: a file-scope device array
// that the code object brings with it on every GPU the library runs on (held
// until the process ends), so a solve through it calls no allocator.
//
// In host code the array's name is only a stand-in for the device symbol; its
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current, and only that address is handed to kernels and copies.

#include <hip/hip_runtime.h>

#include <mutex>

#include "pp_kernels.hpp"

namespace pp {

namespace {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t scratch_buffer(void** ptr) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace pp
