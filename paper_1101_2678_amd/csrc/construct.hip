// construct.hip -- AS tour construction on gfx950 (Section II, Eq. 1; the
// data-parallel design of Section III-A: one workgroup per ant, the ant's
// candidate cities spread over the lanes).
//
// Layout of one step (ant at city `cur`, wavefront of 64 lanes, tile G = 4
// or 8 cities per lane):
//   * the choice row of `cur` is streamed with 16-byte loads; in pass p lane l
//     holds cities 64Gp + Gl .. 64Gp + Gl + G-1, so one pass reads 256 G bytes
//     contiguously and every 64-city block sits in 64/G neighbouring lanes;
//   * visited cities are masked to +0 with a per-lane bit set (bit Gp + e);
//     with SKIP, a 16-byte load whose four cities are all visited (or beyond
//     n) is sent to an out-of-range offset instead, which returns zeros
//     without a memory access, so late in a tour the lines of the row that
//     hold no unvisited city are not fetched at all.  That saves bandwidth
//     where the launch is bandwidth-bound (rows of three or more passes, and
//     the batched launch) but lengthens a step where it is latency-bound
//     (one or two passes with about one wavefront per SIMD), so it is on
//     only in the former;
//   * the total T_b of each 64-city block is a balanced pairwise sum: log2 G
//     levels inside the lane, log2(64/G) DPP levels across the lanes.  That
//     is exactly the last entry of the 64-wide S64 prefix tree, so every T_b
//     is bit-identical to the roulette's definition whatever G is;
//   * T_b move to lane b (a cross-lane read per pass, or for rows of one
//     pass an LDS store and load) and are scanned with S64 (DPP), giving the
//     block offsets E_b and the total;
//   * a block can hold the chosen city only if fl(E_b + T_b (1 + 2^-20)) >
//     target: every inner prefix of a block is at most T_b (1 + 13 u) for a
//     depth-6 tree of non-negative terms (u = 2^-24), so blocks failing this
//     test can be skipped without changing the result;
//   * surviving blocks are rescanned one element per lane with the exact S64
//     tree, in block order, until the first feasible prefix above the target.
// Random numbers: Philox draws (seed, iter, ant, step), 64 steps at a time on
// the vector unit.
#include <type_traits>

#include "r64_lanes.hpp"

namespace aco {
namespace {

constexpr int kSkipOffset = 1 << 30;  // past any row: a buffer load there returns 0

// Per-lane feasibility bits: bit G p + e <=> city 64 G p + G lane + e is < n
// and not yet visited.
template <int G, int P>
__device__ __forceinline__ uint64_t initial_lane_bits(int n, int lane) {
    uint64_t bits = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < G; ++e)
            if (p * Tile<G>::kPass + lane * G + e < n) bits |= 1ull << (p * G + e);
    return bits;
}

// The per-lane feasibility bits in 32 bits where P G <= 32 (rows of up to
// 1024 cities), so that clearing one takes 32-bit operations only.
template <int G, int P>
using LaneBits = std::conditional_t<(P * G <= 32), uint32_t, uint64_t>;

// Marks city j visited in both tabu representations (called with j uniform).
template <int G, typename B>
__device__ __forceinline__ void mark_visited(int j, int lane, B& lane_bits,
                                             uint64_t& block_bits) {
    // j >= 0: unsigned, so the divisions are shifts and masks
    const uint32_t uj = (uint32_t)j;
    if (lane == (int)(uj >> 6)) block_bits |= 1ull << (uj & 63);
    const int owner = (int)((uj % Tile<G>::kPass) / G);
    const int bit = (int)((uj / Tile<G>::kPass) * G + (uj % G));
    // a select rather than a branch around the owner lane
    lane_bits &= lane == owner ? ~((B)1 << bit) : ~(B)0;
}

// Stages the masked weights of block `b` into s_w (city 64b + t at
// s_w[64 (b mod G) + t]).  The block lives in pass b/G, lanes
// (64/G)(b mod G) .. (64/G)(b mod G + 1) - 1; the pass index is wave-uniform
// but not a compile-time constant, so each pass has its own branch, and the
// stores are opaque to the optimiser so that it cannot merge the branches
// into per-register selects.
template <int G, int P>
__device__ __forceinline__ void stage_block(const u32x4 (&wa)[P], const u32x4 (&wb)[P], int b,
                                            float* s_w, int lane) {
    const int pb = b / G;
    if (lane / Tile<G>::kLanesPerBlock != (b % G)) return;
    const uint32_t addr = (uint32_t)(uintptr_t)(s_w + lane * G);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if (p == pb) {
            if (G == 8)
                asm volatile("ds_write_b128 %0, %1\n\tds_write_b128 %0, %2 offset:16"
                             :
                             : "v"(addr), "v"(wa[p]), "v"(wb[p])
                             : "memory");
            else
                asm volatile("ds_write_b128 %0, %1" : : "v"(addr), "v"(wa[p]) : "memory");
        }
    }
}

// Issues the loads of row `row` of the ld-padded matrix `mat` into wa/wb:
// in pass p lane l takes cities 64Gp + Gl .. + G - 1.  The descriptor
// spans `records` bytes from mat and stays the same for the whole tour; the
// row is selected by the scalar offset (two scalar operations per step), and
// the range check covers scalar plus vector offset.  Loads past the end of
// the span return zeros without touching memory; those past the row's n
// cities but inside the span read padding or the next row, and masking
// (whose bits exist only for cities < n) zeroes them.  With SKIP, a 16-byte
// load whose four cities are all visited goes out of range instead.
template <int G, int P, bool SKIP, typename B>
__device__ __forceinline__ void load_row(const float* __restrict__ mat, int records, int row,
                                         int row_bytes, B lane_bits, int lane, u32x4 (&wa)[P],
                                         u32x4 (&wb)[P]) {
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(mat, records);
    const int soff = row * row_bytes;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t bits = (uint32_t)(lane_bits >> (p * G));
        const int off = (p * Tile<G>::kPass + lane * G) * 4;
        const int oa = (!SKIP || (bits & 0xFu)) ? off : kSkipOffset;
        wa[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, oa, soff, 0);
        if (G == 8) {
            const int ob = (!SKIP || (bits & 0xF0u)) ? off + 16 : kSkipOffset;
            wb[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, ob, soff, 0);
        }
    }
}

// Rows of at most 1024 cities: after masking, every pass's weights go to LDS
// (s_w, city c at s_w[c]), so a candidate block is read back with one load
// and nothing is staged on the way to the selection.  Longer rows keep the
// masked weights in registers and stage only the pass of a candidate block.
template <int G, int P>
constexpr bool kWriteAllPasses = (P * Tile<G>::kPass <= 1024);

// One R64 roulette draw over a loaded row of P passes (wa/wb as load_row
// leaves them; masked in place).  block_bits: the visited bits of block b in
// lane b.  Returns the chosen city, or -1 if no city is feasible.
// Wave-uniform.  The workgroup is one wavefront: its LDS operations execute
// in program order, and every LDS access below uses a lane-dependent index,
// so the compiler keeps the order.
template <int G, int P, typename B>
__device__ __forceinline__ int pick_loaded(u32x4 (&wa)[P], u32x4 (&wb)[P], int n, B lane_bits,
                                           uint64_t block_bits, float* s_T, float* s_w, float u,
                                           int lane) {
    constexpr int LPB = Tile<G>::kLanesPerBlock;
    constexpr bool kAll = kWriteAllPasses<G, P>;
    // Block totals to lane b (0 past the row's blocks).  Rows of two or more
    // passes fetch them with one cross-lane read per pass from the last lane
    // of each group (and rows staged whole store their weights afterwards):
    // against a masked LDS store per pass and a load, n = 1000 4%, n = 1500
    // 4.5%, n = 2400 0.8% faster.  Rows of one pass keep the store and load
    // (cross-lane reads measured 6% slower at n = 512).
    constexpr bool kPermute = P >= 2;
    const int nb = (n + 63) >> 6;
    float T = 0.0f;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint32_t bits = (uint32_t)(lane_bits >> (p * G));
        mask4<0>(wa[p], bits);
        float t;
        if (G == 8) {
            mask4<4>(wb[p], bits);
            t = pair_sum4(wa[p]) + pair_sum4(wb[p]);
        } else {
            t = pair_sum4(wa[p]);
        }
        if (kAll && !kPermute) {
            u32x4* dst = reinterpret_cast<u32x4*>(s_w + p * Tile<G>::kPass + lane * G);
            dst[0] = wa[p];
            if (G == 8) dst[1] = wb[p];
        }
        t = group_pairwise<LPB>(t);
        if (kPermute) {
            // block b = pass p, group b mod G
            const float x = __int_as_float(__builtin_amdgcn_ds_bpermute(
                ((lane % G) * LPB + LPB - 1) * 4, __float_as_int(t)));
            T = lane / G == p ? x : T;
        } else if ((lane % LPB) == LPB - 1) {
            s_T[p * G + lane / LPB] = t;
        }
    }
    if (kPermute) {
        if (kAll) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                u32x4* dst = reinterpret_cast<u32x4*>(s_w + p * Tile<G>::kPass + lane * G);
                dst[0] = wa[p];
                if (G == 8) dst[1] = wb[p];
            }
        }
    } else {
        T = s_T[lane];
    }
    // Rows of at most 1024 cities have nb <= 16 blocks, all in row 0 of the
    // block-total scan, which stage B leaves as it is; rows of at most 2^L
    // blocks need only its first L levels.
    float I;
    if constexpr (kAll)
        I = s64_scan_row0_levels<block_scan_levels(P * G)>(T);
    else
        I = s64_scan(T);
    const float total = read_lane(I, nb - 1);
    const float target = u * total;
    const float E = wave_shift_up1(I);
    const float bound = E + T * kBlockSlack;
    uint64_t cand = ballot(bound > target) & (nb >= 64 ? ~0ull : (1ull << nb) - 1ull);
    // Nearly always exactly one candidate block: a single-exit loop, tested
    // at the bottom, so that the usual step runs through without a taken
    // branch.  It goes on while `more` (the remaining candidates, or 0 once
    // the city is found) is not 0, made opaque so that the test stays one
    // compare of a register pair.
    int j = -1;
    if (__builtin_expect(cand != 0, 1)) {
        uint64_t more;
        do {
            const int b = __builtin_ctzll(cand);
            cand &= cand - 1;
            float w;
            if (kAll) {
                w = s_w[b * 64 + lane];
            } else {
                stage_block<G, P>(wa, wb, b, s_w, lane);
                w = s_w[(b % G) * 64 + lane];
            }
            const uint64_t vis = lane_u64(block_bits, b);
            const float s = s64_scan(w);
            const float eb = read_lane(E, b);
            const uint64_t hit = ballot((eb + s) > target) & ~vis;
            if (hit) j = b * 64 + __builtin_ctzll(hit);
            more = hit != 0 ? 0ull : cand;
            __asm__("" : "+s"(more));
        } while (__builtin_expect(more != 0, 0));
    }
    if (__builtin_expect(j >= 0, 1)) return j;
    return pick_fallback(block_bits);
}

template <int G, int P, bool SKIP, typename B>
__device__ __forceinline__ int r64_pick(const float* __restrict__ mat, int records, int row,
                                        int row_bytes, int n, B lane_bits, uint64_t block_bits,
                                        float* s_T, float* s_w, float u, int lane) {
    u32x4 wa[P], wb[P];
    load_row<G, P, SKIP>(mat, records, row, row_bytes, lane_bits, lane, wa, wb);
    return pick_loaded<G, P>(wa, wb, n, lane_bits, block_bits, s_T, s_w, u, lane);
}

// LDS a construction workgroup needs besides the tour.
struct AntShared {
    float w[1024];      // masked weights of rows up to 1024 cities, else a staged pass
    float T[64];        // block totals in block order
};

// The whole tour of ant k of colony c in iteration `iter`: placement, n - 1
// roulette steps, then length, deposit, tour and neighbour tables.
template <int G, int P, bool SKIP, bool LOAD_FIRST>
__device__ __forceinline__ void construct_ant(const Colony& c, int k, uint32_t iter,
                                              uint16_t* s_tour, AntShared& sh) {
    const int lane = threadIdx.x;
    const int n = c.n;
    const int records = n * c.ld * 4;  // the whole n x ld choice matrix
    const PhiloxKey key{(uint32_t)c.seed, (uint32_t)(c.seed >> 32)};

    const int row_bytes = c.ld * 4;
    uint64_t block_bits = initial_block_bits(n, lane);
    sh.T[lane] = 0.0f;
    LaneBits<G, P> lane_bits = (LaneBits<G, P>)initial_lane_bits<G, P>(n, lane);
    __syncthreads();

    const uint32_t x0 = draw(key, iter, (uint32_t)k, 0u);
    int cur = (int)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);

    // LOAD_FIRST: a step's row loads go out as soon as its city is known, and
    // the bookkeeping of that city (tour entry, visited bits) is done while
    // they are in flight.  That shortens launches of one to three passes
    // (n = 100 14%, n = 1000 7%, n = 1500 4% faster) but made the
    // bandwidth-bound four- and five-pass launches (n = 2048, 2400) no
    // faster or up to 1% slower, which keep the bookkeeping first.  With
    // LOAD_FIRST the loads see the visited bits without the step's own city;
    // with SKIP that only loads a quad once more, and masking (which sees
    // it) zeroes the city.
    float u64 = 0.0f;
    if (LOAD_FIRST) {
        for (int step = 1; step < n; ++step) {
            u32x4 wa[P], wb[P];
            load_row<G, P, SKIP>(c.choice, records, cur, row_bytes, lane_bits, lane, wa, wb);
            if (lane == 0) s_tour[step - 1] = (uint16_t)cur;
            mark_visited<G>(cur, lane, lane_bits, block_bits);
            const int slot = (step - 1) & 63;
            if (__builtin_expect(slot == 0, 0))
                u64 = draws64(key, iter, (uint32_t)k, step, lane);
            const float u = read_lane(u64, slot);
            const int j = pick_loaded<G, P>(wa, wb, n, lane_bits, block_bits, sh.T, sh.w, u,
                                            lane);
            // At every step n - step >= 1 cities are unvisited, so j >= 0;
            // the clamp only keeps the LDS indices in range should that
            // ever break.
            cur = j < 0 ? 0 : j;
        }
    } else {
        for (int step = 1; step < n; ++step) {
            if (lane == 0) s_tour[step - 1] = (uint16_t)cur;
            mark_visited<G>(cur, lane, lane_bits, block_bits);
            const int slot = (step - 1) & 63;
            if (__builtin_expect(slot == 0, 0))
                u64 = draws64(key, iter, (uint32_t)k, step, lane);
            const float u = read_lane(u64, slot);
            const int j = r64_pick<G, P, SKIP>(c.choice, records, cur, row_bytes, n, lane_bits,
                                               block_bits, sh.T, sh.w, u, lane);
            cur = j < 0 ? 0 : j;
        }
    }
    if (lane == 0) s_tour[n - 1] = (uint16_t)cur;
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

template <int G, int P>
__global__ __launch_bounds__(64) void k_construct(Colony c, uint32_t iter) {
    extern __shared__ uint16_t s_tour[];
    __shared__ __align__(16) AntShared sh;
    construct_ant<G, P, (P >= 3), (P < 4)>(c, ant_of_block(blockIdx.x, c.m), iter, s_tour, sh);
}

// Batched construction: workgroup g builds ant (antmap[g] & 0xffff) of colony
// cols[antmap[g] >> 16] in that colony's current iteration (*iter_dev).  Each
// colony carries its own tile, and its pass count picks the ant's code
// (batch_ant).  P8 bounds the passes of tile-8 colonies (every colony of the
// launch has n <= 512 P8), so a batch of small instances holds no registers
// for rows it does not have; tile 4 is only ever set for n <= 1024 (4
// passes).
// Loads first in the batched launch too, for rows of one to three passes (as
// in the single-instance launch): 757 -> 764 solves/s on the 256-instance
// workload (n 50..1000, same box).  Longer rows keep the bookkeeping first,
// which is no slower where construction is bound by memory.
template <int NP>
constexpr bool kBatchLoadFirst = NP < 4;

// The ant's code for its colony's exact pass count NP (1 .. PMAX): each
// instance runs a loop specialised for its row length, with no per-pass
// test of the pass count inside the step (256 instances, n 50..1000: 757 ->
// 762 solves/s against one loop with run-time pass tests).
template <int G, int NP, int PMAX>
__device__ __forceinline__ void batch_ant(const Colony& c, int k, uint32_t iter, int np,
                                          uint16_t* s_tour, AntShared& sh) {
    if constexpr (NP < PMAX) {
        if (np != NP) {
            batch_ant<G, NP + 1, PMAX>(c, k, iter, np, s_tour, sh);
            return;
        }
    }
    construct_ant<G, NP, true, kBatchLoadFirst<NP>>(c, k, iter, s_tour, sh);
}

template <int P8>
__global__ __launch_bounds__(64) void k_construct_batch(const Colony* __restrict__ cols,
                                                        const uint32_t* __restrict__ antmap) {
    extern __shared__ uint16_t s_tour[];
    __shared__ __align__(16) AntShared sh;
    const uint32_t e = antmap[blockIdx.x];
    const Colony c = cols[e >> 16];
    // One value for the whole workgroup.  Read through a pointer the kernel
    // might write, it would otherwise be taken as per-lane, and with it the
    // start city and every row address of the tour, each load of which then
    // becomes a loop over lanes.
    const uint32_t iter = __builtin_amdgcn_readfirstlane(*c.iter_dev);
    const int k = (int)(e & 0xffffu);
    if (c.tile == 4) {
        const int np = __builtin_amdgcn_readfirstlane((c.n + 255) / 256);
        batch_ant<4, 1, 4>(c, k, iter, np, s_tour, sh);
    } else {
        const int np = __builtin_amdgcn_readfirstlane((c.n + 511) / 512);
        batch_ant<8, 1, P8>(c, k, iter, np, s_tour, sh);
    }
}

template <int G, int P>
__global__ __launch_bounds__(64) void k_test_select(const float* rows, int ld, int n,
                                                     const uint8_t* feasible, const float* us,
                                                     int32_t* out) {
    __shared__ __align__(16) AntShared sh;
    const int lane = threadIdx.x;
    const int q = blockIdx.x;
    const uint8_t* f = feasible + (size_t)q * n;
    uint64_t vis = ~0ull;
    for (int t = 0; t < 64; ++t) {
        const int j = lane * 64 + t;
        if (j < n && f[j]) vis &= ~(1ull << t);
    }
    sh.T[lane] = 0.0f;
    uint64_t lane_bits = 0;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < G; ++e) {
            const int j = p * Tile<G>::kPass + lane * G + e;
            if (j < n && f[j]) lane_bits |= 1ull << (p * G + e);
        }
    __syncthreads();
    // one row per query: the span is that row's n cities (rounded up to whole
    // 16-byte loads; the caller's padding columns are zero)
    const int j = r64_pick<G, P, true>(rows + (size_t)q * ld, ((n + 3) & ~3) * 4, 0, ld * 4, n,
                                       lane_bits, vis, sh.T, sh.w, us[q], lane);
    if (lane == 0) out[q] = j;
}

// Batched launches can hold at most `wg_per_cu` workgroups on a compute unit
// by asking for more dynamic LDS than the tour needs.  Each workgroup keeps
// one choice row in flight; with more of them the rows evict one another
// from the L2 of each XCD, with fewer the latency of a step is no longer
// covered.  The cap is part of a batch's launch configuration, chosen by the
// batch autotuner; the default (used by the server) caps at 16 per CU, the
// best of a manual sweep on a 256-instance batch (n 50..1000: 18 and 20 were
// 0.7% and 0.6% slower, 24 2.5%, no cap 8.7%, 14 2.1%, 12 13.5%), and only
// launches of at least kCapRounds rounds at the cap: one that fits the
// device in a round or two would only gain a tail.
constexpr int kBatchWgPerCu = 16;
constexpr int kCapRounds = 8;

}  // namespace

size_t batch_lds_bytes(int max_n, int wg_per_cu, size_t lds_per_cu) {
    const size_t tour = tour_lds_bytes(max_n);
    if (wg_per_cu <= 0 || lds_per_cu == 0) return tour;
    const size_t per_wg = lds_per_cu / (size_t)wg_per_cu;
    const size_t fixed = sizeof(AntShared) + 64;  // static LDS and its alignment
    const size_t cap = per_wg > fixed ? (per_wg - fixed) & ~(size_t)255 : 0;
    return tour > cap ? tour : cap;
}

int batch_default_cap(int total_ants, int cus) {
    return total_ants >= kCapRounds * kBatchWgPerCu * cus ? kBatchWgPerCu : 0;
}

namespace {

// Calls f.template operator()<G, P>() for the tile and pass count of n.
template <typename F>
hipError_t dispatch_tile(int tile, int n, F&& f) {
    if (tile == 4) {
        switch ((n + 255) / 256) {
            case 1: return f.template operator()<4, 1>();
            case 2: return f.template operator()<4, 2>();
            case 3: return f.template operator()<4, 3>();
            case 4: return f.template operator()<4, 4>();
            default: return hipErrorInvalidValue;
        }
    }
    switch ((n + 511) / 512) {
        case 1: return f.template operator()<8, 1>();
        case 2: return f.template operator()<8, 2>();
        case 3: return f.template operator()<8, 3>();
        case 4: return f.template operator()<8, 4>();
        case 5: return f.template operator()<8, 5>();
        case 6: return f.template operator()<8, 6>();
        case 7: return f.template operator()<8, 7>();
        case 8: return f.template operator()<8, 8>();
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool tile_supported(int tile, int n) {
    if (tile == 8) return n >= 1 && n <= kMaxCities;
    if (tile == 4) return n >= 1 && n <= 1024;
    return false;
}

int construct_occupancy(const Colony& c) {
    if (c.waves > 1) return construct_split_occupancy(c);
    int blocks = -1;
    (void)dispatch_tile(c.tile, c.n, [&]<int G, int P>() {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_construct<G, P>, 64,
                                                         tour_lds_bytes(c.n)) != hipSuccess)
            blocks = -1;
        return hipSuccess;
    });
    return blocks;
}

hipError_t launch_construct(const Colony& c, uint32_t iter, hipStream_t s) {
    if (c.waves > 1) return launch_construct_split(c, iter, s);
    if (!tile_supported(c.tile, c.n)) return hipErrorInvalidValue;
    return dispatch_tile(c.tile, c.n, [&]<int G, int P>() {
        hipLaunchKernelGGL((k_construct<G, P>), dim3(c.m), dim3(64), tour_lds_bytes(c.n), s, c,
                           iter);
        return hipGetLastError();
    });
}

hipError_t launch_construct_batch(const Colony* cols, const uint32_t* antmap, int total_ants,
                                  int max_n, size_t lds, hipStream_t s) {
    if (total_ants <= 0) return hipSuccess;
    if (max_n < 1 || max_n > kMaxCities) return hipErrorInvalidValue;
    if (lds < tour_lds_bytes(max_n)) return hipErrorInvalidValue;
    const int passes = (max_n + 511) / 512;
    const dim3 grid(total_ants), block(64);
    if (passes <= 2)
        hipLaunchKernelGGL(k_construct_batch<2>, grid, block, lds, s, cols, antmap);
    else if (passes <= 4)
        hipLaunchKernelGGL(k_construct_batch<4>, grid, block, lds, s, cols, antmap);
    else if (passes <= 6)
        hipLaunchKernelGGL(k_construct_batch<6>, grid, block, lds, s, cols, antmap);
    else
        hipLaunchKernelGGL(k_construct_batch<8>, grid, block, lds, s, cols, antmap);
    return hipGetLastError();
}

hipError_t launch_test_select(int tile, int n, int count, const float* rows,
                              const uint8_t* feasible, const float* u, int32_t* out,
                              hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (!tile_supported(tile, n)) return hipErrorInvalidValue;
    const int ld = (n + 63) & ~63;
    return dispatch_tile(tile, n, [&]<int G, int P>() {
        hipLaunchKernelGGL((k_test_select<G, P>), dim3(count), dim3(64), 0, s, rows, ld, n,
                           feasible, u, out);
        return hipGetLastError();
    });
}

}  // namespace aco
