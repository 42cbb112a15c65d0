// Device scratch of the allocation-free entry points: one file-scope device array
// per GPU, found once per device through its symbol address.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kernels.hpp"

namespace lsdd {

// staging for lsdd_elem_bilinear_noalloc: elem_ptr (n_elem + 1 entries) and the
// block offsets (n_elem + 1 entries) of at most NOALLOC_MAX_ELEM elements
static __device__ __align__(256) int64_t scratch[2 * (NOALLOC_MAX_ELEM + 1)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
int64_t* g_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int64_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        // the array's host-side name is not a device address: look it up on this device
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = static_cast<int64_t*>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace lsdd
