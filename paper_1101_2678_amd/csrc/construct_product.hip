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
// multiply throughput rather than by memory.  Each lane keeps only the
// largest product key of each pass (one max per city); a DPP reduction gives
// the wave's largest key, a ballot per pass finds the lowest pass and lane
// holding it, and that lane's lowest position holding it gives the city.
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

// Layout of a row over the W wavefronts of an ant: in pass p, lane l of wave
// w holds cities 512 p + 64 GW w + GW l .. + GW - 1 with GW = 8 / W cities per
// lane, so every 512-city pass is split evenly between the waves and each
// lane's cities are GW / 4 whole Philox blocks.
template <int W>
struct Lay {
    static_assert(W == 1 || W == 2, "one or two wavefronts per ant");
    static constexpr int GW = kG / W;
    __device__ static constexpr int city(int p, int w, int lane, int e) {
        return kPass * p + 64 * GW * w + GW * lane + e;
    }
};

// Draws of one step from Philox for lane `lane` of wave w: block 1 + q + b
// holds cities 4 (q + b) .. + 3 (q = first city / 4).
struct PhiloxDraws {
    uint32_t k0, k1, step, ant, iter;
    template <int P, int W>
    __device__ __forceinline__ void get_all(int w, int lane, float (&r)[P][Lay<W>::GW]) const {
        constexpr int B = Lay<W>::GW / 4;  // blocks per lane per pass
        uint32_t ctr[B * P];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int b = 0; b < B; ++b)
                ctr[B * p + b] = 1u + (uint32_t)Lay<W>::city(p, w, lane, 0) / 4u + (uint32_t)b;
        u32x4 x[B * P];
        philox4_many<B * P>(k0, k1, step, ant, iter, ctr, x);
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e) r[p][4 * b + e] = unit24(x[B * p + b][e]);
    }
};

// Draws given in memory (verification entry point): n floats per row.
struct ArrayDraws {
    const float* u;
    int n;
    template <int P, int W>
    __device__ __forceinline__ void get_all(int w, int lane, float (&r)[P][Lay<W>::GW]) const {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int e = 0; e < Lay<W>::GW; ++e) {
                const int j = Lay<W>::city(p, w, lane, e);
                r[p][e] = j < n ? u[j] : 0.0f;
            }
    }
};

// All ones if bit e of `bits` is set, else 0 (one v_bfe_i32).  Inline
// assembly here: through the builtin the compiler scheduled this kernel 3.5%
// slower (n = 2400), while the roulette kernels gained from it.
__device__ __forceinline__ uint32_t bit_mask(uint32_t bits, int e) {
    uint32_t m;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(m) : "v"(bits), "i"(e));
    return m;
}

// One wave's share of the selection: bit GW p + e of `bits` says whether the
// lane's city e of pass p may be chosen.  Products of finite non-negative
// values are finite and non-negative, so their bit patterns order like the
// values; a city that may not be chosen gets key 0.  Returns the wave's
// largest key and the lowest city holding it; if no product of a city that
// may be chosen is positive, key 0 and the lowest city that may be chosen
// (all products equal, so the lowest index wins); city ~0 if there is none.
struct Pick {
    uint32_t key, city;
};

template <int P, int W, typename Draws>
__device__ __forceinline__ Pick product_pick(const float* row, int n, uint64_t bits,
                                             const Draws& draws, int w, int lane) {
    constexpr int GW = Lay<W>::GW;
    constexpr int L = GW / 4;  // 16-byte loads per lane per pass
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(row), (short)0, ((n + 3) & ~3) * 4, 0x00020000);
    u32x4 wv[P][L];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int b = 0; b < L; ++b)
            wv[p][b] = __builtin_amdgcn_raw_buffer_load_b128(
                rs, (Lay<W>::city(p, w, lane, 0) + 4 * b) * 4, 0, 0);
    // every row load above is in flight before the first draw is computed
    __builtin_amdgcn_sched_barrier(0);
    float r[P][GW];
    draws.template get_all<P, W>(w, lane, r);
    uint32_t key[P][GW], pmax[P];
    uint32_t lmax = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t pass_bits = (uint32_t)(bits >> (GW * p));
        uint32_t m = 0;
#pragma unroll
        for (int e = 0; e < GW; ++e) {
            const float prod = __uint_as_float(wv[p][e / 4][e % 4]) * r[p][e];
            key[p][e] = __float_as_uint(prod) & bit_mask(pass_bits, e);
            m = max(m, key[p][e]);
        }
        pmax[p] = m;
        lmax = max(lmax, m);
    }
    const uint32_t top = wave_max_u32(lmax);
    if (top != 0u) {
        // cities grow with (pass, lane, position): the first pass with a lane
        // holding top, its lowest such lane, that lane's lowest position
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint64_t hold = ballot(pmax[p] == top);
            if (hold) {
                const int src = __builtin_ctzll(hold);
                uint32_t first = 0;
#pragma unroll
                for (int e = GW - 1; e >= 0; --e) first = key[p][e] == top ? (uint32_t)e : first;
                const int e = __builtin_amdgcn_readlane((int)first, src);
                // wave-uniform; said so, or the next row's address is taken
                // as per-lane and every load of it becomes a loop
                const int city = __builtin_amdgcn_readfirstlane(Lay<W>::city(p, w, src, e));
                return Pick{top, (uint32_t)city};
            }
        }
    }
    // No positive product: the lowest city that may be chosen.  Bit GW p + e
    // grows with the city inside a lane.
    uint32_t low = ~0u;
    if (bits) {
        const int b = __builtin_ctzll(bits);
        low = (uint32_t)Lay<W>::city(b / GW, w, lane, b % GW);
    }
    return Pick{0u, wave_min_u32(low)};
}

// Feasibility bits of a fresh tour: cities < n.
template <int P, int W>
__device__ __forceinline__ uint64_t initial_bits(int n, int w, int lane) {
    uint64_t bits = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < Lay<W>::GW; ++e)
            if (Lay<W>::city(p, w, lane, e) < n) bits |= 1ull << (Lay<W>::GW * p + e);
    return bits;
}

// Clears city j's bit in the lane (of the wave) that holds it.
template <int W>
__device__ __forceinline__ void mark_visited(int j, int w, int lane, uint64_t& bits) {
    constexpr uint32_t GW = Lay<W>::GW;
    // j >= 0: unsigned, so the divisions are shifts and masks
    const uint32_t uj = (uint32_t)j;
    const uint32_t p = uj / kPass, rem = uj - p * kPass;
    const uint32_t jw = rem / (64 * GW), r2 = rem - jw * 64 * GW;
    if ((int)jw == w && (int)(r2 / GW) == lane) bits &= ~(1ull << (GW * p + r2 % GW));
}

// Wavefronts per ant of the construction kernel (and of its verification
// entry point).  Two waves per ant double the waves a SIMD can switch
// between but measured no faster: the kernel is bound by the instructions
// it issues (draws and per-city selection), which the split does not
// reduce, so one wave per ant, without a per-step barrier, is the default.
constexpr int kWaves = 1;

template <int P>
__global__ __launch_bounds__(64 * kWaves) void k_construct_product(Colony c, uint32_t iter) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* s_tour = reinterpret_cast<uint16_t*>(smem);
    __shared__ uint32_t s_key[2][kWaves], s_city[2][kWaves];
    __shared__ long long s_len[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int k = ant_of_block(blockIdx.x, c.m);
    const int n = c.n;
    const PhiloxKey key{(uint32_t)c.seed, (uint32_t)(c.seed >> 32)};

    uint64_t bits = initial_bits<P, kWaves>(n, w, lane);
    const uint32_t x0 = draw(key, iter, (uint32_t)k, 0u);
    int cur = (int)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);
    if (tid == 0) s_tour[0] = (uint16_t)cur;
    mark_visited<kWaves>(cur, w, lane, bits);

    for (int step = 1; step < n; ++step) {
        const PhiloxDraws draws{key.k0, key.k1, (uint32_t)step, (uint32_t)k, iter};
        const Pick mine = product_pick<P, kWaves>(c.choice + (size_t)cur * c.ld, n, bits, draws,
                                                  w, lane);
        int next;
        if constexpr (kWaves == 1) {
            next = mine.city == ~0u ? -1 : (int)mine.city;
        } else {
            // winners of both waves, double-buffered by step parity: a wave
            // can rewrite a slot only after passing the next barrier, which
            // the other wave reaches only after reading it
            const int par = step & 1;
            if (lane == 0) {
                s_key[par][w] = mine.key;
                s_city[par][w] = mine.city;
            }
            __syncthreads();
            const uint32_t k0 = s_key[par][0], k1 = s_key[par][1];
            const uint32_t top = k0 > k1 ? k0 : k1;
            const uint32_t c0 = k0 == top ? s_city[par][0] : ~0u;
            const uint32_t c1 = k1 == top ? s_city[par][1] : ~0u;
            const uint32_t j = c0 < c1 ? c0 : c1;
            next = j == ~0u ? -1 : (int)j;
        }
        // n - step >= 1 cities are unvisited, so next >= 0; the clamp only
        // keeps the LDS index in range should that ever break.
        next = next < 0 ? 0 : next;
        if (tid == 0) s_tour[step] = (uint16_t)next;
        mark_visited<kWaves>(next, w, lane, bits);
        cur = next;
    }
    __syncthreads();
    if (tid == 0) s_tour[n] = s_tour[0];
    __syncthreads();

    // Tour length C^k (int64), deposit fl32(1/C^k), tour and neighbour tables.
    long long len = 0;
    for (int s = tid; s < n; s += 64 * kWaves) {
        const int i = s_tour[s], j = s_tour[s + 1];
        len += c.dist[(size_t)i * c.ld + j];
        c.succ[(size_t)i * c.mp + k] = (uint16_t)j;
        c.pred[(size_t)j * c.mp + k] = (uint16_t)i;
    }
    uint16_t* trow = c.tours + (size_t)k * c.tp;
    for (int s = tid; s <= n; s += 64 * kWaves) trow[s] = s_tour[s];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) len += __shfl_xor(len, off);
    if (lane == 0) s_len[w] = len;
    __syncthreads();
    if (tid == 0) {
        long long total = 0;
#pragma unroll
        for (int v = 0; v < kWaves; ++v) total += s_len[v];
        c.lens[k] = total;
        c.dep[k] = (float)(1.0 / (double)total);
    }
}

template <int P>
__global__ __launch_bounds__(64 * kWaves) void k_test_product_select(const float* rows, int ld,
                                                                     int n,
                                                                     const uint8_t* feasible,
                                                                     const float* u, int32_t* out) {
    __shared__ uint32_t s_key[kWaves], s_city[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int q = blockIdx.x;
    const uint8_t* f = feasible + (size_t)q * n;
    uint64_t bits = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < Lay<kWaves>::GW; ++e) {
            const int j = Lay<kWaves>::city(p, w, lane, e);
            if (j < n && f[j]) bits |= 1ull << (Lay<kWaves>::GW * p + e);
        }
    const ArrayDraws draws{u + (size_t)q * n, n};
    const Pick mine = product_pick<P, kWaves>(rows + (size_t)q * ld, n, bits, draws, w, lane);
    if (lane == 0) {
        s_key[w] = mine.key;
        s_city[w] = mine.city;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t top = 0;
        for (int v = 0; v < kWaves; ++v) top = s_key[v] > top ? s_key[v] : top;
        uint32_t j = ~0u;
        for (int v = 0; v < kWaves; ++v)
            if (s_key[v] == top && s_city[v] < j) j = s_city[v];
        out[q] = j == ~0u ? -1 : (int)j;
    }
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
        hipLaunchKernelGGL((k_construct_product<P>), dim3(c.m), dim3(64 * kWaves),
                           tour_bytes(c.n), s, c, iter);
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
        hipLaunchKernelGGL((k_test_product_select<P>), dim3(count), dim3(64 * kWaves), 0, s, rows,
                           ld, n, feasible, u, out);
        return hipGetLastError();
    });
}

}  // namespace aco
