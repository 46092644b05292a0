// The peak search of asp_find_peak for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): no context, no allocation.  Its scratch -- the per-work-group
// packed keys that a context keeps in its device state -- is a file-scope
// device array, one copy per GPU, kept until the process ends.
#include <stdio.h>

#include <mutex>

#include "asp_device.h"
#include "cycle.h"

namespace asp {
namespace {

// The packed keys (|v| bits << 32) | (0xFFFFFFFF - idx), one slot per
// work-group index mod kPeakSlots: 512 bytes per GPU.
__device__ __align__(256) unsigned long long scratch[kPeakSlots];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
unsigned long long *g_scratch[kMaxDevices];   // device address of `scratch` per GPU

__global__ void k_na_clear(unsigned long long *slots)
{
    if (threadIdx.x < kPeakSlots) slots[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void k_na_scan(const float *__restrict__ R, int64_t n,
                                                 unsigned long long *slots)
{
    peak_scan(R, n, blockIdx.x, gridDim.x, slots);
}

// One wave: the maximum over the slots, decoded into the pixel index and the
// residual value there.
__global__ void k_na_out(const float *__restrict__ R, const unsigned long long *slots,
                         int64_t *idx_out, float *value_out)
{
    unsigned long long k = __hip_atomic_load(&slots[threadIdx.x], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(k, off, 64);
        k = o > k ? o : k;
    }
    if (threadIdx.x == 0) {
        const int64_t idx = (int64_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
        *idx_out = idx;
        *value_out = R[idx];
    }
}

// The device address of `scratch` on the current GPU, resolved once per GPU.
hipError_t scratch_on_device(unsigned long long **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_lock);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<unsigned long long *>(ptr);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace asp

extern "C" asp_status asp_find_peak_noalloc(const float *R, int64_t H, int64_t W,
                                            int64_t *idx_out, float *value_out, void *stream)
{
    if (!R || !idx_out || !value_out || H <= 0 || W <= 0) return ASP_ERR_INVALID_ARG;
    if ((double)H * (double)W >= 4294967295.0) {
        fprintf(stderr, "asp_find_peak_noalloc: %lld x %lld pixels exceed the maximum of "
                        "2^32 - 2 (the packed key holds a 32-bit index)\n",
                (long long)H, (long long)W);
        return ASP_ERR_INVALID_ARG;
    }
    if (reinterpret_cast<uintptr_t>(R) % 16 != 0) {
        fprintf(stderr, "asp_find_peak_noalloc: the image must be 16-byte aligned\n");
        return ASP_ERR_INVALID_ARG;
    }
    unsigned long long *slots = nullptr;
    if (asp::scratch_on_device(&slots) != hipSuccess) return ASP_ERR_DEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess) return ASP_ERR_DEVICE;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t n = H * W;
    const int64_t need = (n / 4 + 255) / 256;
    const int64_t cap = 8 * (int64_t)cus;
    const int grid = (int)(need < 1 ? 1 : (need < cap ? need : cap));
    hipLaunchKernelGGL(asp::k_na_clear, dim3(1), dim3(asp::kPeakSlots), 0, s, slots);
    hipLaunchKernelGGL(asp::k_na_scan, dim3(grid), dim3(256), 0, s, R, n, slots);
    hipLaunchKernelGGL(asp::k_na_out, dim3(1), dim3(asp::kPeakSlots), 0, s, R,
                       (const unsigned long long *)slots, idx_out, value_out);
    return hipGetLastError() == hipSuccess ? ASP_OK : ASP_ERR_DEVICE;
}
