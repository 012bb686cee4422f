// Library-held scratch memory for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).  One file-scope device
// array serves every such call on a device; each device that loads the library holds its own
// copy until the process ends.
//
// In host code the array's name is only a host-side handle: its device address is taken once
// per device with hipGetSymbolAddress (with that device current, from hough_config) and every
// later use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hough_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[hough::kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Zero fill: a kernel rather than a memset node, so that the same code stays safe wherever a
// caller's stream may be captured.
__global__ __launch_bounds__(256) void k_zero(uint4 *p, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

namespace hough {

// Called with `device` current.  Takes the array's device address and zero-fills it once per
// device (the split form's kernels then keep it zero between calls).
int scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return HOUGH_EDEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return HOUGH_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HOUGH_EDEVICE;
    static_assert(kStaticScratchBytes % 16 == 0, "whole 16-byte words");
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, (hipStream_t)0, static_cast<uint4 *>(ptr),
                       kStaticScratchBytes / 16);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize((hipStream_t)0) != hipSuccess)
        return HOUGH_EDEVICE;
    g_ptr[device] = ptr;
    return HOUGH_OK;
}

void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace hough
