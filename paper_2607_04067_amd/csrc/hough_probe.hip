// Measurement probe of libhough_probe.so: the LDS atomic rate of the access pattern the vote
// kernels use, so that a benchmark can state its LDS-atomic ceiling from a live measurement on
// the machine it runs on instead of a constant.
//
// Pattern (the packed tile of the vote kernels): a tile of R rows of 32 dwords in LDS; lane l of
// a wave adds 1 << (16 * (l >> 5)) to dword 32 * row + (l & 31), so the 64 lanes touch 32
// consecutive dwords of one row, the two lanes of a dword in different halves of the wave (no
// bank conflict, no same-address collision within a half).  Each wave walks rows with an odd
// stride (a different row per instruction, as the votes of successive hits do), eight atomics in
// flight between the address updates.  Nothing else runs in the loop: the rate is the LDS's.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kRows = 256;

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_lds_add(int iters, uint32_t *sink) {
    __shared__ uint32_t tile[kRows * 32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kRows * 32; i += NW * 64) tile[i] = 0u;
    __syncthreads();
    const uint32_t inc = 1u << (16 * (lane >> 5));
    const uint32_t col = (uint32_t)(lane & 31);
    uint32_t row = (uint32_t)(wave * 29 + blockIdx.x * 7) & (kRows - 1);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t r = (row + 37u * (uint32_t)u) & (kRows - 1);
            __hip_atomic_fetch_add(&tile[r * 32 + col], inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        row = (row + 11u) & (kRows - 1);
    }
    __syncthreads();
    // one word per workgroup keeps the loop from being removed
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int i = 0; i < 32; ++i) s += tile[i];
        sink[blockIdx.x] = s;
    }
}

template <int NW>
hipError_t launch(int blocks, int iters, uint32_t *sink, hipStream_t s) {
    hipLaunchKernelGGL(k_lds_add<NW>, dim3(blocks), dim3(NW * 64), 0, s, iters, sink);
    return hipGetLastError();
}

}  // namespace

extern "C" {

// Lane-updates one launch performs: blocks * waves * 64 * iters * 8.
// blocks: workgroups (a multiple of the CU count fills the chip evenly); waves: 4, 8 or 16 per
// workgroup; iters >= 1; sink: device buffer of `blocks` uint32.  Returns 0, -1 for a bad
// argument, -4 for a launch failure.
int hough_probe_lds_add(int blocks, int waves, int iters, uint32_t *sink, void *stream) {
    if (blocks < 1 || iters < 1 || !sink) return -1;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    switch (waves) {
        case 4: e = launch<4>(blocks, iters, sink, s); break;
        case 8: e = launch<8>(blocks, iters, sink, s); break;
        case 16: e = launch<16>(blocks, iters, sink, s); break;
        default: return -1;
    }
    return e == hipSuccess ? 0 : -4;
}

}  // extern "C"
