// Scratch memory of lmep_step_noalloc: a static array in every device's
// memory that the library owns, for callers that cannot allocate device memory
// or hand over a workspace; plus the kernel that writes a call's problem tables
// into it from kernel arguments, so that such a call needs no host staging
// buffer either.
#include <cstring>
#include <mutex>

#include "lmep_internal.hpp"

namespace lmep {

// Held by every device the library runs on until the process ends.  In host
// code this name stands for a host-side shadow, not for device memory: the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_mu;
void* g_ptr[64] = {};

// 4-byte words carried in the kernel arguments of one launch.
constexpr int kArgWords = 768;
struct ArgWords {
    int32_t count;
    uint32_t w[kArgWords];
};

__global__ __launch_bounds__(256) void copy_words_kernel(uint32_t* __restrict__ dst, ArgWords src) {
    for (int i = threadIdx.x; i < src.count; i += blockDim.x) dst[i] = src.w[i];
}

}  // namespace

hipError_t static_scratch(void** d_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *d_out = g_ptr[dev];
    return hipSuccess;
}

hipError_t upload_by_args(void* d_dst, const void* host, size_t bytes, hipStream_t stream) {
    if (bytes % 4 != 0 || ((uintptr_t)d_dst) % 4 != 0) return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    ArgWords a;
    for (size_t done = 0; done < words; done += kArgWords) {
        const size_t k = words - done < (size_t)kArgWords ? words - done : (size_t)kArgWords;
        a.count = (int32_t)k;
        std::memcpy(a.w, (const char*)host + 4 * done, 4 * k);
        hipLaunchKernelGGL(copy_words_kernel, dim3(1), dim3(256), 0, stream, (uint32_t*)d_dst + done, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lmep
