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

// Streaming read of a buffer `reps` times.  The buffer is cut into chunks of
// 256 threads x L loads of 16 bytes, all L in flight before any is used
// (NT: nontemporal loads, which do not keep the lines in the caches).
// Workgroups go to the eight XCDs round-robin by index, so work item w runs
// on XCD w mod 8; XCD x walks the whole buffer chunk by chunk, starting x/8
// of the way in.  Every XCD's L2 therefore sees the whole footprint cycling
// through it, as in tour construction, where every XCD reads rows from the
// whole choice matrix: a footprint above the L2 is served from the Infinity
// Cache (MALL) or HBM, one below it from the L2.  The sum keeps the loads
// alive and goes to sink[blockIdx.x].
constexpr int kStreamThreads = 256;

template <int L, bool NT>
__global__ __launch_bounds__(kStreamThreads) void k_probe_read(const float4* __restrict__ src,
                                                               size_t n16, size_t chunks,
                                                               size_t items, float* sink) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    constexpr size_t kChunk16 = (size_t)kStreamThreads * L;  // 16-byte units
    float acc = 0.0f;
    for (size_t w = blockIdx.x; w < items; w += gridDim.x) {
        const size_t x = w & 7, k = w >> 3;
        const size_t c = (k + x * (chunks / 8 + 1)) % chunks;
        const size_t base = c * kChunk16 + threadIdx.x;
        f4v v[L];
#pragma unroll
        for (int u = 0; u < L; ++u) {
            const size_t i = base + (size_t)u * kStreamThreads;
            const f4v* p = reinterpret_cast<const f4v*>(src + i);
            if (i < n16)
                v[u] = NT ? __builtin_nontemporal_load(p) : *p;
            else
                v[u] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int u = 0; u < L; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    __shared__ float red[kStreamThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kStreamThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

constexpr int kProbeBlocks = 4096;

// Random-row read probe: the memory access pattern of tour construction
// without its arithmetic.  One wavefront per workgroup reads `steps` whole
// rows of `row_len` floats (row pitch `ld`), lane l taking 8 consecutive
// floats per 512-float pass; the row of step s is a hash of (workgroup, s), so
// consecutive rows of one wavefront, and the rows of different wavefronts,
// are independent and uniformly spread over `rows`.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

typedef unsigned int probe_u32x4 __attribute__((ext_vector_type(4)));

// R rows in flight per wavefront: the loads of R consecutive steps' rows are
// issued before any of them is used.
template <int P, int R>
__global__ __launch_bounds__(64) void k_probe_rows(const float* mat, int rows, int ld,
                                                   int row_len, int steps, float* sink) {
    const int lane = threadIdx.x;
    uint32_t acc = 0;
    for (int s0 = 0; s0 < steps; s0 += R) {
        probe_u32x4 a[R][P], b[R][P];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int s = s0 + q < steps ? s0 + q : steps - 1;
            const uint32_t h = mix32((uint32_t)blockIdx.x * 0x9E3779B9u + (uint32_t)s);
            const int r = (int)(((uint64_t)h * (uint32_t)rows) >> 32);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float*>(mat + (size_t)r * ld), (short)0, ((row_len + 3) & ~3) * 4,
                0x00020000);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int off = (p * 512 + lane * 8) * 4;
                a[q][p] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
                b[q][p] = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int p = 0; p < P; ++p)
                acc ^= a[q][p].x ^ a[q][p].y ^ a[q][p].z ^ a[q][p].w ^ b[q][p].x ^ b[q][p].y ^
                       b[q][p].z ^ b[q][p].w;
    }
    if (acc == 0x12345678u) sink[blockIdx.x] = 1.0f;  // keeps the loads alive
}

template <int R>
hipError_t launch_probe_rows_r(const float* mat, int rows, int ld, int row_len, int waves,
                               int steps, float* sink, hipStream_t s) {
    const dim3 g(waves), b(64);
    switch ((row_len + 511) / 512) {
        case 1: hipLaunchKernelGGL((k_probe_rows<1, R>), g, b, 0, s, mat, rows, ld, row_len, steps, sink); break;
        case 2: hipLaunchKernelGGL((k_probe_rows<2, R>), g, b, 0, s, mat, rows, ld, row_len, steps, sink); break;
        case 3: hipLaunchKernelGGL((k_probe_rows<3, R>), g, b, 0, s, mat, rows, ld, row_len, steps, sink); break;
        case 4: hipLaunchKernelGGL((k_probe_rows<4, R>), g, b, 0, s, mat, rows, ld, row_len, steps, sink); break;
        case 5: hipLaunchKernelGGL((k_probe_rows<5, R>), g, b, 0, s, mat, rows, ld, row_len, steps, sink); break;
        case 6: hipLaunchKernelGGL((k_probe_rows<6, R>), g, b, 0, s, mat, rows, ld, row_len, steps, sink); break;
        case 7: hipLaunchKernelGGL((k_probe_rows<7, R>), g, b, 0, s, mat, rows, ld, row_len, steps, sink); break;
        case 8: hipLaunchKernelGGL((k_probe_rows<8, R>), g, b, 0, s, mat, rows, ld, row_len, steps, sink); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_probe_rows(const float* mat, int rows, int ld, int row_len, int waves,
                             int steps, int rows_in_flight, float* sink, hipStream_t s) {
    if (waves <= 0 || steps <= 0) return hipSuccess;
    if (rows_in_flight == 1) return launch_probe_rows_r<1>(mat, rows, ld, row_len, waves, steps, sink, s);
    if (rows_in_flight == 2) return launch_probe_rows_r<2>(mat, rows, ld, row_len, waves, steps, sink, s);
    return hipErrorInvalidValue;
}

hipError_t launch_probe_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    const int blocks = (int)((n16 + 255) / 256 < (size_t)kProbeBlocks ? (n16 + 255) / 256
                                                                        : (size_t)kProbeBlocks);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<float4*>(dst), reinterpret_cast<const float4*>(src), n16);
    return hipGetLastError();
}

template <int L, bool NT>
hipError_t launch_probe_read_shape(const void* src, size_t bytes, int reps, float* sink,
                                   hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0 || reps <= 0) return hipSuccess;
    // chunks * reps work items in all, so each XCD walks the whole buffer
    // reps / 8 times; the grid is a multiple of 8 workgroups (or one work item
    // per workgroup), so work item w always runs on XCD w mod 8.
    constexpr size_t kChunk16 = (size_t)kStreamThreads * L;
    const size_t chunks = (n16 + kChunk16 - 1) / kChunk16;
    const size_t items = chunks * (size_t)reps;
    const int blocks = (int)(items < (size_t)kProbeBlocks ? items : (size_t)kProbeBlocks);
    hipLaunchKernelGGL((k_probe_read<L, NT>), dim3(blocks), dim3(kStreamThreads), 0, s,
                       reinterpret_cast<const float4*>(src), n16, chunks, items, sink);
    return hipGetLastError();
}

hipError_t launch_probe_read(const void* src, size_t bytes, int reps, int loads, bool nontemporal,
                             float* sink, hipStream_t s) {
    switch (loads * 2 + (nontemporal ? 1 : 0)) {
        case 8: return launch_probe_read_shape<4, false>(src, bytes, reps, sink, s);
        case 9: return launch_probe_read_shape<4, true>(src, bytes, reps, sink, s);
        case 16: return launch_probe_read_shape<8, false>(src, bytes, reps, sink, s);
        case 17: return launch_probe_read_shape<8, true>(src, bytes, reps, sink, s);
        case 32: return launch_probe_read_shape<16, false>(src, bytes, reps, sink, s);
        case 33: return launch_probe_read_shape<16, true>(src, bytes, reps, sink, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace aco
