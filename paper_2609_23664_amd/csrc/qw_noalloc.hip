// Fixed device scratch of the allocation-free sampler entry point
// (qw_sample_noalloc): a file-scope device array that every GPU the library
// runs on holds until the process ends, looked up once per device.
//
// In host code the array's name is not a device address; host code only
// ever uses the address that hipGetSymbolAddress returns for the current
// device (noalloc_scratch below).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "qw_kernels.h"

namespace qw {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Slot pointers of `count` slots of `stride` bytes from `base`.
__global__ __launch_bounds__(256) void slot_ptrs_kernel(const float2 **out, const char *base,
                                                        uint64_t stride, uint32_t count) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = reinterpret_cast<const float2 *>(base + (uint64_t)i * stride);
}

}  // namespace

hipError_t noalloc_scratch(int device, void **ptr) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = p;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

hipError_t launch_slot_ptrs(hipStream_t st, const float2 **out, const void *base, uint64_t stride,
                            uint32_t count) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(slot_ptrs_kernel, dim3((count + 255) / 256), dim3(256), 0, st, out,
                       static_cast<const char *>(base), stride, count);
    return hipGetLastError();
}

}  // namespace qw
