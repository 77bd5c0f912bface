// Device scratch of the allocation-free reductions.
//
// pss_structure_factor allocates its shell accumulators on first use
// (hipMalloc).  Callers that cannot allocate device memory use
// pss_structure_factor_noalloc, whose partial results live in the file-scope
// array below instead.  Every GPU that the library runs on holds its own copy
// of the array until the process ends, and every call on that GPU shares it:
// calls that overlap on one GPU race.
//
// In host code the name `scratch` is a host-side stand-in, not a device
// address; host code only ever uses the address hipGetSymbolAddress returns
// for the current device, cached per device below.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pss_kernels.h"

namespace pss {

// room for the accumulators of kScratchShells shells (kShellWords 64-bit
// words each: 128-bit sum, count, exponent key): 64 KiB
static __device__ __align__(256) unsigned long long scratch[kScratchShells * kShellWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

__global__ void zero_words_kernel(unsigned long long* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}
}  // namespace

hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        // once per device, with that device current: its copy of the array
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return hipSuccess;
}

hipError_t launch_zero_words(hipStream_t s, unsigned long long* p, int n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_words_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace pss
