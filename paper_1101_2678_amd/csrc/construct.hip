// construct.hip -- AS tour construction on gfx950 (Section II, Eq. 1; the
// data-parallel design of Section III-A: one workgroup per ant, the ant's
// candidate cities spread over the lanes).
//
// Layout of one step (ant at city `cur`, wavefront of 64 lanes):
//   * the choice row of `cur` is streamed with 16-byte loads; in pass p lane l
//     holds cities 512p + 8l .. 512p + 8l + 7, so one pass reads 2 KB
//     contiguously and every 64-city block sits in 8 neighbouring lanes;
//   * visited cities are masked to +0 with a per-lane bit set (bit 8p + e);
//   * the total T_b of each 64-city block is a balanced pairwise sum: three
//     levels inside the lane, three DPP levels across the 8 lanes.  That is
//     exactly the last entry of the 64-wide S64 prefix tree, so every T_b is
//     bit-identical to the roulette's definition;
//   * T_b move to lane b through LDS and are scanned with S64 (DPP), giving
//     the block offsets E_b and the total;
//   * a block can hold the chosen city only if fl(E_b + T_b (1 + 2^-20)) >
//     target: every inner prefix of a block is at most T_b (1 + 13 u) for a
//     depth-6 tree of non-negative terms (u = 2^-24), so blocks failing this
//     test can be skipped without changing the result;
//   * surviving blocks are rescanned one element per lane with the exact S64
//     tree, in block order, until the first feasible prefix above the target.
// Random numbers: Philox draw (seed, iter, ant, step) on the scalar unit.
#include "aco_device.hpp"
#include "aco_state.hpp"

namespace aco {
namespace {

constexpr float kBlockSlack = 1.00000095367431640625f;  // 1 + 2^-20

// Per-lane feasibility bits: bit 8p + e <=> city 512p + 8 lane + e is < n and
// not yet visited.
template <int P>
__device__ __forceinline__ uint64_t initial_lane_bits(int n, int lane) {
    uint64_t bits = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < kCitiesPerLane; ++e)
            if (p * kPassCities + lane * kCitiesPerLane + e < n) bits |= 1ull << (p * 8 + e);
    return bits;
}

// s_vis[b]: bit t set <=> city 64b + t is visited or does not exist.
__device__ __forceinline__ uint64_t initial_block_bits(int n, int b) {
    const int valid = n - 64 * b;
    if (valid <= 0) return ~0ull;
    if (valid >= 64) return 0ull;
    return ~0ull << valid;
}

// Clears city j in both tabu representations (called with j uniform).
__device__ __forceinline__ void mark_visited(int j, int lane, uint64_t& lane_bits,
                                             uint64_t* s_vis) {
    if (lane == 0)
        __hip_atomic_fetch_or(&s_vis[j >> 6], 1ull << (j & 63), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_WORKGROUP);
    const int owner = (j & (kPassCities - 1)) >> 3;
    const int bit = ((j / kPassCities) << 3) + (j & 7);
    if (lane == owner) lane_bits &= ~(1ull << bit);
}

// Buffer view of one choice row: loads at or beyond `valid_bytes` return 0
// without touching memory.  valid_bytes is n rounded up to 4 cities, so a
// 16-byte load is either wholly inside or wholly outside the row; the padding
// columns between n and that bound hold zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float* row, int valid_bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(row), (short)0, valid_bytes,
                                             0x00020000);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Sign-extended bit `e` of `bits` (0 or all ones).  Written as v_bfe_i32 so
// the masking of one city costs two VALU operations (extract, and).
template <int E>
__device__ __forceinline__ uint32_t bit_mask(uint32_t bits) {
    uint32_t m;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(m) : "v"(bits), "i"(E));
    return m;
}

// Stages the masked weights of block `b` into s_w (city 64b + t at
// s_w[64 (b mod 8) + t]).  The block lives in pass b/8, lanes 8 (b mod 8) ..
// 8 (b mod 8) + 7; the pass index is wave-uniform but not a compile-time
// constant, so each pass has its own branch, and the stores are opaque to the
// optimiser so that it cannot merge the branches into per-register selects.
template <int P>
__device__ __forceinline__ void stage_block(const u32x4 (&wa)[P], const u32x4 (&wb)[P], int b,
                                            float* s_w, int lane) {
    const int pb = b >> 3;
    if ((lane >> 3) != (b & 7)) return;
    const uint32_t addr = (uint32_t)(uintptr_t)(s_w + lane * kCitiesPerLane);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (p == pb) {
            asm volatile("ds_write_b128 %0, %1\n\tds_write_b128 %0, %2 offset:16"
                         :
                         : "v"(addr), "v"(wa[p]), "v"(wb[p])
                         : "memory");
        }
    }
}

// One R64 roulette draw over `row` (ld-padded, zero beyond n).
// Returns the chosen city, or -1 if no city is feasible.  Wave-uniform.
// The masked weights stay in registers; the pass holding a candidate block
// is staged into LDS (city j at s_w[j]) only when that block is scanned.  The
// workgroup is one wavefront: its LDS operations execute in program order,
// and every LDS access below uses a lane-dependent index, so the compiler
// keeps the order.
template <int P>
__device__ __forceinline__ int r64_pick(const float* __restrict__ row, int n, uint64_t lane_bits,
                                        const uint64_t* s_vis, float* s_T, float* s_w, float u,
                                        int lane) {
    const int nb = (n + 63) >> 6;
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(row, ((n + 3) & ~3) * 4);
    u32x4 wa[P], wb[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int off = (p * kPassCities + lane * kCitiesPerLane) * 4;
        wa[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        wb[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t bits = (uint32_t)(lane_bits >> (p * 8));
        wa[p].x &= bit_mask<0>(bits);
        wa[p].y &= bit_mask<1>(bits);
        wa[p].z &= bit_mask<2>(bits);
        wa[p].w &= bit_mask<3>(bits);
        wb[p].x &= bit_mask<4>(bits);
        wb[p].y &= bit_mask<5>(bits);
        wb[p].z &= bit_mask<6>(bits);
        wb[p].w &= bit_mask<7>(bits);
        float t = ((__uint_as_float(wa[p].x) + __uint_as_float(wa[p].y)) +
                   (__uint_as_float(wa[p].z) + __uint_as_float(wa[p].w))) +
                  ((__uint_as_float(wb[p].x) + __uint_as_float(wb[p].y)) +
                   (__uint_as_float(wb[p].z) + __uint_as_float(wb[p].w)));
        t = octet_pairwise(t);
        if ((lane & 7) == 7) s_T[p * 8 + (lane >> 3)] = t;
    }
    const float T = s_T[lane];
    const float I = s64_scan(T);
    const float total = read_lane(I, nb - 1);
    const float target = u * total;
    const float E = wave_shift_up1(I);
    const float bound = E + T * kBlockSlack;
    uint64_t cand = ballot(lane < nb && bound > target);
    while (cand) {
        const int b = __builtin_ctzll(cand);
        cand &= cand - 1;
        stage_block<P>(wa, wb, b, s_w, lane);
        const uint64_t vis = s_vis[b];
        const float w = s_w[(b & 7) * 64 + lane];
        const bool feasible = ((vis >> lane) & 1ull) == 0ull;
        const float s = s64_scan(w);
        const float eb = read_lane(E, b);
        const uint64_t hit = ballot(feasible && (eb + s) > target);
        if (hit) return b * 64 + __builtin_ctzll(hit);
    }
    // No prefix exceeds the target: the highest feasible city.
    const uint64_t live = ballot(~s_vis[lane] != 0ull);
    if (!live) return -1;
    const int b = 63 - __builtin_clzll(live);
    return b * 64 + 63 - __builtin_clzll(~s_vis[b]);
}

// Uniform draws for steps s0 .. s0+63: lane t holds u of step s0 + t.  The
// counter words differ per lane, so the ten Philox rounds run on the vector
// unit once per 64 steps instead of on the scalar unit every step.
__device__ __forceinline__ float draws64(PhiloxKey key, uint32_t iter, uint32_t ant, int s0,
                                         int lane) {
    return uniform24(draw(key, iter, ant, (uint32_t)(s0 + lane)));
}

template <int P>
__global__ __launch_bounds__(64) void k_construct(Colony c, uint32_t iter) {
    extern __shared__ uint16_t s_tour[];
    __shared__ __align__(16) float s_w[kPassCities];
    __shared__ uint64_t s_vis[64];
    __shared__ float s_T[64];
    const int lane = threadIdx.x;
    const int k = blockIdx.x;
    const int n = c.n;
    const PhiloxKey key{(uint32_t)c.seed, (uint32_t)(c.seed >> 32)};

    s_vis[lane] = initial_block_bits(n, lane);
    s_T[lane] = 0.0f;
    uint64_t lane_bits = initial_lane_bits<P>(n, lane);
    __syncthreads();

    const uint32_t x0 = draw(key, iter, (uint32_t)k, 0u);
    int cur = (int)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);
    if (lane == 0) s_tour[0] = (uint16_t)cur;
    mark_visited(cur, lane, lane_bits, s_vis);

    float u64 = 0.0f;
    for (int step = 1; step < n; ++step) {
        const int slot = (step - 1) & 63;
        if (slot == 0) u64 = draws64(key, iter, (uint32_t)k, step, lane);
        const float u = read_lane(u64, slot);
        const float* row = c.choice + (size_t)cur * c.ld;
        int j = r64_pick<P>(row, n, lane_bits, s_vis, s_T, s_w, u, lane);
        // At every step n - step >= 1 cities are unvisited, so j >= 0; the
        // clamp only keeps the LDS indices in range should that ever break.
        j = j < 0 ? 0 : j;
        if (lane == 0) s_tour[step] = (uint16_t)j;
        mark_visited(j, lane, lane_bits, s_vis);
        cur = j;
    }
    __syncthreads();
    if (lane == 0) s_tour[n] = s_tour[0];
    __syncthreads();

    // Tour length C^k (int64), deposit fl32(1/C^k), tour and neighbour tables.
    long long len = 0;
    for (int s = lane; s < n; s += 64) {
        const int i = s_tour[s], j = s_tour[s + 1];
        len += c.dist[(size_t)i * c.ld + j];
        c.succ[(size_t)i * c.mp + k] = (uint16_t)j;
        c.pred[(size_t)j * c.mp + k] = (uint16_t)i;
    }
    uint16_t* trow = c.tours + (size_t)k * c.tp;
    for (int s = lane; s <= n; s += 64) trow[s] = s_tour[s];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) len += __shfl_xor(len, off);
    if (lane == 0) {
        c.lens[k] = len;
        c.dep[k] = (float)(1.0 / (double)len);
    }
}

template <int P>
__global__ __launch_bounds__(64) void k_test_select(const float* rows, int ld, int n,
                                                     const uint8_t* feasible, const float* us,
                                                     int32_t* out) {
    __shared__ __align__(16) float s_w[kPassCities];
    __shared__ uint64_t s_vis[64];
    __shared__ float s_T[64];
    const int lane = threadIdx.x;
    const int q = blockIdx.x;
    const uint8_t* f = feasible + (size_t)q * n;
    uint64_t vis = ~0ull;
    for (int t = 0; t < 64; ++t) {
        const int j = lane * 64 + t;
        if (j < n && f[j]) vis &= ~(1ull << t);
    }
    s_vis[lane] = vis;
    s_T[lane] = 0.0f;
    uint64_t lane_bits = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < kCitiesPerLane; ++e) {
            const int j = p * kPassCities + lane * kCitiesPerLane + e;
            if (j < n && f[j]) lane_bits |= 1ull << (p * 8 + e);
        }
    __syncthreads();
    const int j =
        r64_pick<P>(rows + (size_t)q * ld, n, lane_bits, s_vis, s_T, s_w, us[q], lane);
    if (lane == 0) out[q] = j;
}

template <int P>
hipError_t launch_construct_p(const Colony& c, uint32_t iter, hipStream_t s) {
    const size_t lds = ((size_t)(c.n + 1) * sizeof(uint16_t) + 15) & ~(size_t)15;
    hipLaunchKernelGGL(k_construct<P>, dim3(c.m), dim3(64), lds, s, c, iter);
    return hipGetLastError();
}

template <int P>
hipError_t launch_select_p(int n, int count, const float* rows, const uint8_t* feasible,
                           const float* u, int32_t* out, hipStream_t s) {
    const int ld = (n + 63) & ~63;
    hipLaunchKernelGGL(k_test_select<P>, dim3(count), dim3(64), 0, s, rows, ld, n, feasible, u,
                       out);
    return hipGetLastError();
}

template <int P>
int occupancy_p(const Colony& c) {
    int blocks = 0;
    const size_t lds = ((size_t)(c.n + 1) * sizeof(uint16_t) + 15) & ~(size_t)15;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_construct<P>, 64, lds) !=
        hipSuccess)
        return -1;
    return blocks;
}

}  // namespace

int construct_occupancy(const Colony& c) {
    switch ((c.n + kPassCities - 1) / kPassCities) {
        case 1: return occupancy_p<1>(c);
        case 2: return occupancy_p<2>(c);
        case 3: return occupancy_p<3>(c);
        case 4: return occupancy_p<4>(c);
        case 5: return occupancy_p<5>(c);
        case 6: return occupancy_p<6>(c);
        case 7: return occupancy_p<7>(c);
        case 8: return occupancy_p<8>(c);
        default: return -1;
    }
}

hipError_t launch_construct(const Colony& c, uint32_t iter, hipStream_t s) {
    switch ((c.n + kPassCities - 1) / kPassCities) {
        case 1: return launch_construct_p<1>(c, iter, s);
        case 2: return launch_construct_p<2>(c, iter, s);
        case 3: return launch_construct_p<3>(c, iter, s);
        case 4: return launch_construct_p<4>(c, iter, s);
        case 5: return launch_construct_p<5>(c, iter, s);
        case 6: return launch_construct_p<6>(c, iter, s);
        case 7: return launch_construct_p<7>(c, iter, s);
        case 8: return launch_construct_p<8>(c, iter, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_test_select(int n, int count, const float* rows, const uint8_t* feasible,
                              const float* u, int32_t* out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch ((n + kPassCities - 1) / kPassCities) {
        case 1: return launch_select_p<1>(n, count, rows, feasible, u, out, s);
        case 2: return launch_select_p<2>(n, count, rows, feasible, u, out, s);
        case 3: return launch_select_p<3>(n, count, rows, feasible, u, out, s);
        case 4: return launch_select_p<4>(n, count, rows, feasible, u, out, s);
        case 5: return launch_select_p<5>(n, count, rows, feasible, u, out, s);
        case 6: return launch_select_p<6>(n, count, rows, feasible, u, out, s);
        case 7: return launch_select_p<7>(n, count, rows, feasible, u, out, s);
        case 8: return launch_select_p<8>(n, count, rows, feasible, u, out, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace aco
