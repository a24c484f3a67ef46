// construct_product.hip -- tour construction with the paper's data-parallel
// selection (Section III-A; Table II, versions 7-8): every unvisited city j of
// the current row draws its own uniform r_j, the product fl32(choice[i][j] *
// r_j) is formed, and the largest product wins (lowest j among equal ones).
// Visited cities are left out of the reduction rather than multiplied by 0,
// and the tile winners compete on the same product, so the tiling of the row
// over lanes cannot change the result.
//
// r_j = (x >> 8) * 2^-24 with x = word (j mod 4) of Philox4x32-10 at counter
// (step, ant, iter, 1 + j / 4), key = seed: one Philox block serves four
// consecutive cities.
//
// One wavefront per ant; in pass p lane l holds cities 512 p + 8 l .. +7 (two
// 16-byte loads of the choice row, two Philox blocks).  All loads of a step
// are issued before the first Philox block is computed, so the row streams
// while the vector unit generates the draws; per step the kernel does n / 4
// Philox blocks per ant and reads 4n bytes, which makes it bound by integer
// multiply throughput rather than by memory.  Each lane keeps its first
// maximum in increasing city order; two DPP reductions (largest product key,
// then lowest city among the lanes holding it) give the next city.
#include <hip/hip_runtime.h>

#include "aco_device.hpp"
#include "aco_state.hpp"
#include "product.hpp"

namespace aco {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kG = 8;              // cities per lane per pass
constexpr int kPass = 64 * kG;     // cities per pass
constexpr int kMaxPasses = kMaxCities / kPass;

size_t tour_bytes(int n) { return ((size_t)(n + 1) * sizeof(uint16_t) + 15) & ~(size_t)15; }

// a ^ b ^ k in one v_bitop3_b32 (truth table 0x96); k is wave-uniform.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "s"(k));
    return d;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), all four output words.
// The 32 x 32 -> 64-bit products give both halves in one multiply.  With
// only the last counter word varying across lanes, part of rounds 1-3 is
// wave-uniform and the compiler keeps it on the scalar unit; from round 3
// on every value varies per lane and the two XORs of a word fuse into one
// three-input operation.
// NB Philox blocks that differ only in the last counter word, computed round
// by round across the blocks: NB independent multiply chains per round keep
// the vector unit busy although a SIMD holds only two or three ants.
template <int NB>
__device__ __forceinline__ void philox4_many(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                             uint32_t c2, const uint32_t (&c3)[NB],
                                             u32x4 (&out)[NB]) {
    uint32_t a[NB], b[NB], c[NB], d[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        a[i] = c0;
        b[i] = c1;
        c[i] = c2;
        d[i] = c3[i];
    }
#pragma unroll
    for (int r = 0; r < 10; ++r) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const uint64_t pa = (uint64_t)0xD2511F53u * a[i];
            const uint64_t pb = (uint64_t)0xCD9E8D57u * c[i];
            uint32_t y0, y2;
            if (r >= 3) {
                y0 = xor3((uint32_t)(pb >> 32), b[i], k0);
                y2 = xor3((uint32_t)(pa >> 32), d[i], k1);
            } else {
                y0 = (uint32_t)(pb >> 32) ^ b[i] ^ k0;
                y2 = (uint32_t)(pa >> 32) ^ d[i] ^ k1;
            }
            a[i] = y0;
            b[i] = (uint32_t)pb;
            c[i] = y2;
            d[i] = (uint32_t)pa;
        }
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) out[i] = u32x4{a[i], b[i], c[i], d[i]};
}

__device__ __forceinline__ float unit24(uint32_t x) { return (float)(x >> 8) * 0x1.0p-24f; }

template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, kCtrl, kRowMask, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    x = max(x, dpp_u32<0x111, 0xF>(0u, x));
    x = max(x, dpp_u32<0x112, 0xF>(0u, x));
    x = max(x, dpp_u32<0x114, 0xF>(0u, x));
    x = max(x, dpp_u32<0x118, 0xF>(0u, x));
    x = max(x, dpp_u32<0x142, 0xA>(0u, x));
    x = max(x, dpp_u32<0x143, 0xC>(0u, x));
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
    x = min(x, dpp_u32<0x111, 0xF>(~0u, x));
    x = min(x, dpp_u32<0x112, 0xF>(~0u, x));
    x = min(x, dpp_u32<0x114, 0xF>(~0u, x));
    x = min(x, dpp_u32<0x118, 0xF>(~0u, x));
    x = min(x, dpp_u32<0x142, 0xA>(~0u, x));
    x = min(x, dpp_u32<0x143, 0xC>(~0u, x));
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Draws of one step from Philox: lane l's eight cities of every pass p
// (blocks 1 + q and 2 + q, q = (512 p + 8 l) / 4).
struct PhiloxDraws {
    uint32_t k0, k1, step, ant, iter;
    template <int P>
    __device__ __forceinline__ void get_all(int lane, float (&r)[P][kG]) const {
        uint32_t ctr[2 * P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t q = (uint32_t)(kPass * p + kG * lane) / 4u;
            ctr[2 * p] = 1u + q;
            ctr[2 * p + 1] = 2u + q;
        }
        u32x4 x[2 * P];
        philox4_many<2 * P>(k0, k1, step, ant, iter, ctr, x);
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                r[p][e] = unit24(x[2 * p][e]);
                r[p][4 + e] = unit24(x[2 * p + 1][e]);
            }
    }
};

// Draws given in memory (verification entry point): n floats per row.
struct ArrayDraws {
    const float* u;
    int n;
    template <int P>
    __device__ __forceinline__ void get_all(int lane, float (&r)[P][kG]) const {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int e = 0; e < kG; ++e) {
                const int j = kPass * p + kG * lane + e;
                r[p][e] = j < n ? u[j] : 0.0f;
            }
    }
};

// All ones if bit e of `bits` is set, else 0 (one v_bfe_i32).
__device__ __forceinline__ uint32_t bit_mask(uint32_t bits, int e) {
    uint32_t m;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(m) : "v"(bits), "i"(e));
    return m;
}

// The next city: bit kG p + e of `bits` says whether city 512 p + 8 lane + e
// may be chosen.  Products of finite non-negative values are finite and
// non-negative, so their bit patterns order like the values; key = bits + 1
// (0 = no candidate in this lane).  Returns -1 if no city is feasible.
template <int P, typename Draws>
__device__ __forceinline__ int product_pick(const float* row, int n, uint64_t bits,
                                            const Draws& draws, int lane) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(row), (short)0, ((n + 3) & ~3) * 4, 0x00020000);
    u32x4 wa[P], wb[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int off = (kPass * p + kG * lane) * 4;
        wa[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        wb[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0);
    }
    // every row load above is in flight before the first draw is computed
    __builtin_amdgcn_sched_barrier(0);
    float r[P][kG];
    draws.template get_all<P>(lane, r);
    uint32_t best = 0, best_j = ~0u;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t w[kG] = {wa[p].x, wa[p].y, wa[p].z, wa[p].w,
                                wb[p].x, wb[p].y, wb[p].z, wb[p].w};
        const uint32_t pass_bits = (uint32_t)(bits >> (kG * p));
#pragma unroll
        for (int e = 0; e < kG; ++e) {
            const float prod = __uint_as_float(w[e]) * r[p][e];
            const uint32_t key = (__float_as_uint(prod) + 1u) & bit_mask(pass_bits, e);
            if (key > best) {
                best = key;
                best_j = (uint32_t)(kPass * p + kG * lane + e);
            }
        }
    }
    const uint32_t top = wave_max_u32(best);
    const uint32_t j = wave_min_u32(best == top && best != 0u ? best_j : ~0u);
    return top == 0u ? -1 : (int)j;
}

// Feasibility bits of a fresh tour: cities < n.
template <int P>
__device__ __forceinline__ uint64_t initial_bits(int n, int lane) {
    uint64_t bits = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < kG; ++e)
            if (kPass * p + kG * lane + e < n) bits |= 1ull << (kG * p + e);
    return bits;
}

// Clears city j's bit in the lane that holds it.
__device__ __forceinline__ void mark_visited(int j, int lane, uint64_t& bits) {
    const int p = j / kPass, rem = j - p * kPass;
    if (rem / kG == lane) bits &= ~(1ull << (kG * p + rem % kG));
}

template <int P>
__global__ __launch_bounds__(64) void k_construct_product(Colony c, uint32_t iter) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* s_tour = reinterpret_cast<uint16_t*>(smem);
    const int lane = threadIdx.x;
    const int k = blockIdx.x;
    const int n = c.n;
    const PhiloxKey key{(uint32_t)c.seed, (uint32_t)(c.seed >> 32)};

    uint64_t bits = initial_bits<P>(n, lane);
    const uint32_t x0 = draw(key, iter, (uint32_t)k, 0u);
    int cur = (int)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);
    if (lane == 0) s_tour[0] = (uint16_t)cur;
    mark_visited(cur, lane, bits);

    for (int step = 1; step < n; ++step) {
        const PhiloxDraws draws{key.k0, key.k1, (uint32_t)step, (uint32_t)k, iter};
        int next = product_pick<P>(c.choice + (size_t)cur * c.ld, n, bits, draws, lane);
        // n - step >= 1 cities are unvisited, so next >= 0; the clamp only
        // keeps the LDS index in range should that ever break.
        next = next < 0 ? 0 : next;
        if (lane == 0) s_tour[step] = (uint16_t)next;
        mark_visited(next, lane, bits);
        cur = next;
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
__global__ __launch_bounds__(64) void k_test_product_select(const float* rows, int ld, int n,
                                                            const uint8_t* feasible,
                                                            const float* u, int32_t* out) {
    const int lane = threadIdx.x;
    const int q = blockIdx.x;
    const uint8_t* f = feasible + (size_t)q * n;
    uint64_t bits = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < kG; ++e) {
            const int j = kPass * p + kG * lane + e;
            if (j < n && f[j]) bits |= 1ull << (kG * p + e);
        }
    const ArrayDraws draws{u + (size_t)q * n, n};
    const int j = product_pick<P>(rows + (size_t)q * ld, n, bits, draws, lane);
    if (lane == 0) out[q] = j;
}

// Philox throughput probe: the draws of `steps` steps of a 2400-city row
// (ten blocks per lane per step, the formulation construction uses) without
// loads or selection.  The XOR of all words goes to sink[64 * wave + lane].
__global__ __launch_bounds__(64) void k_probe_philox(int steps, uint32_t seed, uint32_t* sink) {
    const int lane = threadIdx.x;
    uint32_t acc = 0;
    for (int step = 1; step <= steps; ++step) {
        uint32_t ctr[10];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const uint32_t q = (uint32_t)(kPass * i + kG * lane) / 4u;
            ctr[2 * i] = 1u + q;
            ctr[2 * i + 1] = 2u + q;
        }
        u32x4 x[10];
        philox4_many<10>(seed, 0u, (uint32_t)step, blockIdx.x, 0u, ctr, x);
#pragma unroll
        for (int i = 0; i < 10; ++i) acc ^= x[i].x ^ x[i].y ^ x[i].z ^ x[i].w;
    }
    sink[(size_t)blockIdx.x * 64 + lane] = acc;
}

// Calls f.template operator()<P>() for P = ceil(n / 512) in 1..8.
template <int P = 1, typename F>
hipError_t dispatch_passes(int n, F&& f) {
    if constexpr (P > kMaxPasses) {
        return hipErrorInvalidValue;
    } else {
        if ((n + kPass - 1) / kPass == P) return f.template operator()<P>();
        return dispatch_passes<P + 1>(n, f);
    }
}

}  // namespace

hipError_t launch_construct_product(const Colony& c, uint32_t iter, hipStream_t s) {
    if (c.n < 1 || c.n > kMaxCities) return hipErrorInvalidValue;
    return dispatch_passes(c.n, [&]<int P>() {
        hipLaunchKernelGGL((k_construct_product<P>), dim3(c.m), dim3(64), tour_bytes(c.n), s, c,
                           iter);
        return hipGetLastError();
    });
}

hipError_t launch_probe_philox(int waves, int steps, uint32_t seed, uint32_t* sink,
                               hipStream_t s) {
    if (waves <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_philox, dim3(waves), dim3(64), 0, s, steps, seed, sink);
    return hipGetLastError();
}

hipError_t launch_test_product_select(int n, int count, const float* rows,
                                      const uint8_t* feasible, const float* u, int32_t* out,
                                      hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (n < 1 || n > kMaxCities) return hipErrorInvalidValue;
    const int ld = (n + 63) & ~63;
    return dispatch_passes(n, [&]<int P>() {
        hipLaunchKernelGGL((k_test_product_select<P>), dim3(count), dim3(64), 0, s, rows, ld, n,
                           feasible, u, out);
        return hipGetLastError();
    });
}

}  // namespace aco
