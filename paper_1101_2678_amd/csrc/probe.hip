// probe.hip -- bandwidth probes: a plain copy of known traffic (to calibrate
// hardware byte counters) and a repeated streaming read (to measure the read
// bandwidth a footprint achieves, on-die caches included).
#include "aco_device.hpp"
#include "aco_state.hpp"

namespace aco {
namespace {

__global__ __launch_bounds__(256) void k_probe_copy(float4* __restrict__ dst,
                                                    const float4* __restrict__ src, size_t n16) {
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

// Each workgroup streams its share of the buffer `reps` times; the sum keeps
// the loads alive and goes to sink[blockIdx.x].
__global__ __launch_bounds__(256) void k_probe_read(const float4* __restrict__ src, size_t n16,
                                                    int reps, float* sink) {
    const size_t stride = (size_t)gridDim.x * 256;
    float acc = 0.0f;
    for (int r = 0; r < reps; ++r)
        for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) {
            const float4 v = src[i];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    __shared__ float red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

constexpr int kProbeBlocks = 4096;

}  // namespace

hipError_t launch_probe_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    const int blocks = (int)((n16 + 255) / 256 < (size_t)kProbeBlocks ? (n16 + 255) / 256
                                                                        : (size_t)kProbeBlocks);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<float4*>(dst), reinterpret_cast<const float4*>(src), n16);
    return hipGetLastError();
}

hipError_t launch_probe_read(const void* src, size_t bytes, int reps, float* sink,
                             hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0 || reps <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_read, dim3(kProbeBlocks), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(src), n16, reps, sink);
    return hipGetLastError();
}

}  // namespace aco
