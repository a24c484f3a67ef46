// r64_lanes.hpp -- pieces of the R64 roulette step shared by the
// construction kernels with one and with several wavefronts per ant: the
// tile of cities per lane, the masking of visited cities, the in-lane and
// cross-lane pairwise block sums, the per-block visited bits, the buffer view
// of a choice row and the per-step uniform draws (Section II, Eq. 1).
#pragma once

#include "aco_device.hpp"
#include "aco_state.hpp"

namespace aco {
namespace {

constexpr float kBlockSlack = 1.00000095367431640625f;  // 1 + 2^-20
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Cities per lane per pass (G), and what follows from it.
template <int G>
struct Tile {
    static_assert(G == 4 || G == 8, "tile must be 4 or 8 cities per lane");
    static constexpr int kPass = 64 * G;          // cities per pass
    static constexpr int kLanesPerBlock = 64 / G; // lanes holding one 64-city block
};

// Visited bits of block b, kept in lane b of a register pair: bit t set <=>
// city 64b + t is visited or does not exist.
__device__ __forceinline__ uint64_t initial_block_bits(int n, int b) {
    const int valid = n - 64 * b;
    if (valid <= 0) return ~0ull;
    if (valid >= 64) return 0ull;
    return ~0ull << valid;
}

// The value lane l holds in v, on every lane (l wave-uniform).
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Scan levels that cover the block totals of a row of at most `blocks`
// 64-city blocks (at most 16: the blocks sit in row 0 of the scan).
constexpr int block_scan_levels(int blocks) {
    return blocks <= 2 ? 1 : blocks <= 4 ? 2 : blocks <= 8 ? 3 : 4;
}

// No prefix exceeds the target (rounding, or every weight zero): the highest
// feasible city, or -1 if there is none.
__device__ __forceinline__ int pick_fallback(uint64_t block_bits) {
    const uint64_t live = ballot(~block_bits != 0ull);
    if (!live) return -1;
    const int b = 63 - __builtin_clzll(live);
    return b * 64 + 63 - __builtin_clzll(~lane_u64(block_bits, b));
}

// Buffer view of `bytes` bytes from `base`: a load whose scalar plus vector
// offset is at or beyond it returns 0 without touching memory.  Every span
// used is a multiple of 16 bytes, so a 16-byte load is wholly inside or
// wholly outside it.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, bytes,
                                             0x00020000);
}

// Sign-extended bit `e` of `bits` (0 or all ones): one v_bfe_i32, so the
// masking of one city costs two VALU operations (extract, and).  Through the
// builtin rather than inline assembly, so the compiler sees the dependences
// and can extract every mask before the row's loads return.
template <int E>
__device__ __forceinline__ uint32_t bit_mask(uint32_t bits) {
    return (uint32_t)__builtin_amdgcn_sbfe((int)bits, E, 1);
}

template <int E0>
__device__ __forceinline__ void mask4(u32x4& v, uint32_t bits) {
    v.x &= bit_mask<E0 + 0>(bits);
    v.y &= bit_mask<E0 + 1>(bits);
    v.z &= bit_mask<E0 + 2>(bits);
    v.w &= bit_mask<E0 + 3>(bits);
}

__device__ __forceinline__ float pair_sum4(const u32x4& v) {
    return (__uint_as_float(v.x) + __uint_as_float(v.y)) +
           (__uint_as_float(v.z) + __uint_as_float(v.w));
}

// Balanced pairwise sum over groups of LANES consecutive lanes (LANES = 8 or
// 16, inside one 16-lane DPP row); the last lane of each group ends with it.
template <int LANES>
__device__ __forceinline__ float group_pairwise(float x) {
    x = x + dpp_move<0x111, 0xF>(x);
    x = x + dpp_move<0x112, 0xF>(x);
    x = x + dpp_move<0x114, 0xF>(x);
    if (LANES == 16) x = x + dpp_move<0x118, 0xF>(x);
    return x;
}

// Uniform draws for steps s0 .. s0+63: lane t holds u of step s0 + t.  The
// counter words differ per lane, so the ten Philox rounds run on the vector
// unit once per 64 steps instead of on the scalar unit every step.
__device__ __forceinline__ float draws64(PhiloxKey key, uint32_t iter, uint32_t ant, int s0,
                                         int lane) {
    return uniform24(draw(key, iter, ant, (uint32_t)(s0 + lane)));
}

__host__ __device__ size_t tour_lds_bytes(int n) {
    return ((size_t)(n + 1) * sizeof(uint16_t) + 15) & ~(size_t)15;
}

}  // namespace
}  // namespace aco
