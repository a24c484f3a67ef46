// aco_device.hpp -- device building blocks shared by the libaco kernels.
//
// Everything here is written for gfx950 (CDNA4): 64-lane wavefronts, DPP
// row/broadcast moves, scalar unit for wave-uniform integer work.
// Compile with -ffp-contract=off: every floating-point expression below is
// meant to round once per operation, exactly as written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aco {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor bijection with a Weyl-bumped key.  All inputs are
// wave-uniform in every caller, so the compiler keeps this on the scalar
// unit (s_mul_i32 / s_mul_hi_u32).
// ---------------------------------------------------------------------------
struct PhiloxKey {
    uint32_t k0, k1;
};

__device__ __forceinline__ uint32_t philox_word0(PhiloxKey key, uint32_t c0, uint32_t c1,
                                                  uint32_t c2, uint32_t c3) {
    constexpr uint32_t kMulLo = 0xD2511F53u;   // applied to counter word 0
    constexpr uint32_t kMulHi = 0xCD9E8D57u;   // applied to counter word 2
    constexpr uint32_t kBump0 = 0x9E3779B9u;   // golden-ratio Weyl step
    constexpr uint32_t kBump1 = 0xBB67AE85u;   // sqrt(3)-1 Weyl step
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo_a = kMulLo * c0, hi_a = __umulhi(kMulLo, c0);
        const uint32_t lo_b = kMulHi * c2, hi_b = __umulhi(kMulHi, c2);
        const uint32_t y0 = hi_b ^ c1 ^ k0;
        const uint32_t y2 = hi_a ^ c3 ^ k1;
        c0 = y0;
        c1 = lo_b;
        c2 = y2;
        c3 = lo_a;
        k0 += kBump0;
        k1 += kBump1;
    }
    return c0;
}

// Draw for (iter, ant, step): counter (step, ant, iter, 0).
__device__ __forceinline__ uint32_t draw(PhiloxKey key, uint32_t iter, uint32_t ant,
                                         uint32_t step) {
    return philox_word0(key, step, ant, iter, 0u);
}

__device__ __forceinline__ float uniform24(uint32_t x0) {
    return (float)(x0 >> 8) * 0x1.0p-24f;
}

// ---------------------------------------------------------------------------
// DPP helpers.  dpp_ctrl encodings (GFX9): row_shr:k = 0x110 + k,
// wave_shr:1 = 0x138, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
// Lanes whose source is outside the row, or whose row is masked off, get
// `old` = +0, so "x + moved" adds +0 there (exact for x >= +0).
// ---------------------------------------------------------------------------
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_move(float x) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, kRowMask, 0xF, false));
}

// S64: inclusive FP32 prefix over the 64 lanes with a fixed tree.
//   stage A: Kogge-Stone inside each 16-lane row, shifts 1, 2, 4, 8;
//   stage B: row_bcast:15 into rows 1 and 3 (adds R0 resp. R2), then
//            row_bcast:31 into rows 2 and 3 (adds X = R1 + R0).
// The result is independent of how cities were mapped to lanes upstream.
__device__ __forceinline__ float s64_scan(float x) {
    x = x + dpp_move<0x111, 0xF>(x);
    x = x + dpp_move<0x112, 0xF>(x);
    x = x + dpp_move<0x114, 0xF>(x);
    x = x + dpp_move<0x118, 0xF>(x);
    x = x + dpp_move<0x142, 0xA>(x);
    x = x + dpp_move<0x143, 0xC>(x);
    return x;
}

// The first L levels of stage A (L = 1..4).  On lanes 0 .. 2^L - 1 of
// non-negative values this equals s64_scan (stage B leaves row 0 as it is,
// and the later levels of stage A would add +0 there, their source lane
// being below 0, which changes no value >= +0).
template <int L>
__device__ __forceinline__ float s64_scan_row0_levels(float x) {
    static_assert(L >= 1 && L <= 4, "one to four levels");
    x = x + dpp_move<0x111, 0xF>(x);
    if (L >= 2) x = x + dpp_move<0x112, 0xF>(x);
    if (L >= 3) x = x + dpp_move<0x114, 0xF>(x);
    if (L >= 4) x = x + dpp_move<0x118, 0xF>(x);
    return x;
}

// Lane l receives lane l-1's value, lane 0 receives +0.
__device__ __forceinline__ float wave_shift_up1(float x) { return dpp_move<0x138, 0xF>(x); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Workgroups go to the eight XCDs round-robin by index.  A construction
// workgroup b builds ant ant_of_block(b, m), so that each XCD runs one
// contiguous range of ants: the successor and predecessor entries of
// neighbouring ants share cache lines, which are then written from one L2
// instead of in eight partial copies.  A bijection on [0, m); which workgroup
// builds an ant does not change its tour.
__device__ __forceinline__ int ant_of_block(int b, int m) {
    const int x = b & 7, j = b >> 3, q = m >> 3, r = m & 7;
    return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ float read_lane(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// ---------------------------------------------------------------------------
// Heuristic and choice (Eq. 1 numerator): heur = fl32(1 / d^beta) with the
// power by left-to-right binary64 products; zero on the diagonal (d = 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float heur_of(int32_t d, int beta) {
    if (d == 0) return 0.0f;
    double p = 1.0;
    for (int b = 0; b < beta; ++b) p = p * (double)d;
    return (float)(1.0 / p);
}

__device__ __forceinline__ float choice_of(float tau, float heur, int alpha) {
    const float tp = (alpha == 0) ? 1.0f : (alpha == 1 ? tau : tau * tau);
    return tp * heur;
}

}  // namespace aco
