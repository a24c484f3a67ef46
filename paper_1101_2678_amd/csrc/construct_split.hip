// construct_split.hip -- AS tour construction with several wavefronts per
// ant, for rows of at most 1024 cities (Section II, Eq. 1; the ant's cities
// spread over the threads of its block, Section III-A).
//
// With one wavefront per ant and about one ant per SIMD (n = m = 1000 on 256
// compute units), a step is a chain of dependent operations that no other
// wavefront hides.  Here W wavefronts share an ant and split the loading,
// masking and block sums of each row: wave w takes passes w, w + W, ... of
// the single-wave layout (at most PW of them).  Every wave writes its masked
// weights and block totals to LDS, one barrier joins them, and then every
// wave runs the same selection on the same LDS data, so all of them arrive
// at the same city without a second barrier.  The LDS buffers alternate with
// the step's parity: a wave can rewrite a buffer only after the next
// barrier, which the other waves reach only after they have read it.  Block
// totals, block bound and rescan are those of the single-wave kernel, so the
// tours are the same bit for bit.
#include "r64_lanes.hpp"

namespace aco {
namespace {

struct AntSharedSplit {
    float w[2][1024];   // masked weights by step parity, city c at w[.][c]
    float T[2][64];     // block totals by step parity
    long long len[4];   // per-wave partial tour lengths
};

// Lane bits of wave wv: bit G q + e <=> city 64 G (wv + W q) + G lane + e is
// < n and not yet visited.
template <int G, int W, int PW>
__device__ __forceinline__ uint64_t initial_lane_bits_split(int n, int wv, int lane) {
    uint64_t bits = 0;
#pragma unroll
    for (int q = 0; q < PW; ++q)
#pragma unroll
        for (int e = 0; e < G; ++e)
            if ((wv + W * q) * Tile<G>::kPass + lane * G + e < n) bits |= 1ull << (q * G + e);
    return bits;
}

// Marks city j visited: its block bit in every wave, its lane bit in the wave
// holding its pass (called with j and wv wave-uniform).
template <int G, int W>
__device__ __forceinline__ void mark_visited_split(int j, int wv, int lane, uint64_t& lane_bits,
                                                   uint64_t& block_bits) {
    // j >= 0: unsigned, so the divisions are shifts and masks
    const uint32_t uj = (uint32_t)j;
    if (lane == (int)(uj >> 6)) block_bits |= 1ull << (uj & 63);
    const uint32_t p = uj / Tile<G>::kPass;
    const int owner = (int)((uj % Tile<G>::kPass) / G);
    const int bit = (int)((p / W) * G + (uj % G));
    lane_bits &= ((int)(p % W) == wv && lane == owner) ? ~(1ull << bit) : ~0ull;
}

// One R64 draw by the W waves of the workgroup over a row loaded with
// load_split; s_T and s_w are this step's buffers.  Returns the chosen city
// (the same in every wave), or -1 if no city is feasible.
// The wave's passes of row `row` of the ld-padded matrix `mat`, through a
// descriptor spanning `records` bytes and the scalar row offset, as in the
// single-wave kernel (past the span: zeros; past n inside it: masked).
template <int G, int W, int PW>
__device__ __forceinline__ void load_split(const float* __restrict__ mat, int records, int row,
                                           int ld, int np, int wv, int lane, u32x4 (&wa)[PW],
                                           u32x4 (&wb)[PW]) {
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(mat, records);
    const int soff = row * ld * 4;
#pragma unroll
    for (int q = 0; q < PW; ++q) {
        const int p = wv + W * q;
        if (p >= np) break;
        const int off = (p * Tile<G>::kPass + lane * G) * 4;
        wa[q] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, soff, 0);
        if (G == 8) wb[q] = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, soff, 0);
    }
}

// wa/wb as load_split leaves them (masked in place).
template <int G, int W, int PW>
__device__ __forceinline__ int pick_split(u32x4 (&wa)[PW], u32x4 (&wb)[PW], int n, int np,
                                          int wv, uint64_t lane_bits, uint64_t block_bits,
                                          float* s_T, float* s_w, float u, int lane) {
    constexpr int LPB = Tile<G>::kLanesPerBlock;
#pragma unroll
    for (int q = 0; q < PW; ++q) {
        const int p = wv + W * q;
        if (p >= np) break;
        const uint32_t bits = (uint32_t)(lane_bits >> (q * G));
        mask4<0>(wa[q], bits);
        float t;
        if (G == 8) {
            mask4<4>(wb[q], bits);
            t = pair_sum4(wa[q]) + pair_sum4(wb[q]);
        } else {
            t = pair_sum4(wa[q]);
        }
        u32x4* dst = reinterpret_cast<u32x4*>(s_w + p * Tile<G>::kPass + lane * G);
        dst[0] = wa[q];
        if (G == 8) dst[1] = wb[q];
        t = group_pairwise<LPB>(t);
        if ((lane % LPB) == LPB - 1) s_T[p * G + lane / LPB] = t;
    }
    __syncthreads();
    // n <= 1024: at most 16 blocks, all in row 0 of the block-total scan.
    const int nb = (n + 63) >> 6;
    const float T = s_T[lane];
    const float I = s64_scan_row0_levels<block_scan_levels(W * PW * G)>(T);
    const float total = read_lane(I, nb - 1);
    const float target = u * total;
    const float E = wave_shift_up1(I);
    const float bound = E + T * kBlockSlack;
    uint64_t cand = ballot(bound > target) & ((1ull << nb) - 1ull);
    // as in the single-wave kernel: one bottom-tested loop, rarely repeated
    int j = -1;
    if (__builtin_expect(cand != 0, 1)) {
        do {
            const int b = __builtin_ctzll(cand);
            cand &= cand - 1;
            const float w = s_w[b * 64 + lane];
            const uint64_t vis = lane_u64(block_bits, b);
            const float s = s64_scan(w);
            const float eb = read_lane(E, b);
            const uint64_t hit = ballot((eb + s) > target) & ~vis;
            if (hit) j = b * 64 + __builtin_ctzll(hit);
        } while (__builtin_expect(j < 0 && cand != 0, 0));
    }
    if (__builtin_expect(j >= 0, 1)) return j;
    return pick_fallback(block_bits);
}

template <int G, int W, int PW>
__global__ __launch_bounds__(64 * W) void k_construct_split(Colony c, uint32_t iter) {
    extern __shared__ uint16_t s_tour[];
    __shared__ __align__(16) AntSharedSplit sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int k = ant_of_block(blockIdx.x, c.m);
    const int n = c.n;
    const int np = (n + Tile<G>::kPass - 1) / Tile<G>::kPass;
    const PhiloxKey key{(uint32_t)c.seed, (uint32_t)(c.seed >> 32)};

    uint64_t block_bits = initial_block_bits(n, lane);
    uint64_t lane_bits = initial_lane_bits_split<G, W, PW>(n, wv, lane);
    // block totals beyond the row's blocks are never written; keep them finite
    if (tid < 128) sh.T[tid >> 6][lane] = 0.0f;
    __syncthreads();

    const uint32_t x0 = draw(key, iter, (uint32_t)k, 0u);
    int cur = (int)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);

    // As in the single-wave kernel: a step's row loads go out first, the
    // bookkeeping of its city follows them.
    float u64 = 0.0f;
    for (int step = 1; step < n; ++step) {
        u32x4 wa[PW], wb[PW];
        load_split<G, W, PW>(c.choice, n * c.ld * 4, cur, c.ld, np, wv, lane, wa, wb);
        if (tid == 0) s_tour[step - 1] = (uint16_t)cur;
        mark_visited_split<G, W>(cur, wv, lane, lane_bits, block_bits);
        const int slot = (step - 1) & 63;
        if (__builtin_expect(slot == 0, 0)) u64 = draws64(key, iter, (uint32_t)k, step, lane);
        const float u = read_lane(u64, slot);
        const int buf = step & 1;
        const int j = pick_split<G, W, PW>(wa, wb, n, np, wv, lane_bits, block_bits, sh.T[buf],
                                           sh.w[buf], u, lane);
        // n - step >= 1 cities are unvisited, so j >= 0; the clamp only keeps
        // the LDS indices in range should that ever break.
        cur = j < 0 ? 0 : j;
    }
    if (tid == 0) s_tour[n - 1] = (uint16_t)cur;
    __syncthreads();
    if (tid == 0) s_tour[n] = s_tour[0];
    __syncthreads();

    long long len = 0;
    for (int s = tid; s < n; s += 64 * W) {
        const int i = s_tour[s], j = s_tour[s + 1];
        len += c.dist[(size_t)i * c.ld + j];
        c.succ[(size_t)i * c.mp + k] = (uint16_t)j;
        c.pred[(size_t)j * c.mp + k] = (uint16_t)i;
    }
    uint16_t* trow = c.tours + (size_t)k * c.tp;
    for (int s = tid; s <= n; s += 64 * W) trow[s] = s_tour[s];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) len += __shfl_xor(len, off);
    if (lane == 0) sh.len[wv] = len;
    __syncthreads();
    if (tid == 0) {
        long long total = 0;
#pragma unroll
        for (int v = 0; v < W; ++v) total += sh.len[v];
        c.lens[k] = total;
        c.dep[k] = (float)(1.0 / (double)total);
    }
}

// One selection per workgroup by W waves, for the verification entry point.
template <int G, int W, int PW>
__global__ __launch_bounds__(64 * W) void k_test_select_split(const float* rows, int ld, int n,
                                                              const uint8_t* feasible,
                                                              const float* us, int32_t* out) {
    __shared__ __align__(16) AntSharedSplit sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = blockIdx.x;
    const uint8_t* f = feasible + (size_t)q * n;
    const int np = (n + Tile<G>::kPass - 1) / Tile<G>::kPass;
    uint64_t vis = ~0ull;
    for (int t = 0; t < 64; ++t) {
        const int j = lane * 64 + t;
        if (j < n && f[j]) vis &= ~(1ull << t);
    }
    uint64_t lane_bits = 0;
#pragma unroll
    for (int r = 0; r < PW; ++r)
#pragma unroll
        for (int e = 0; e < G; ++e) {
            const int j = (wv + W * r) * Tile<G>::kPass + lane * G + e;
            if (j < n && f[j]) lane_bits |= 1ull << (r * G + e);
        }
    if (tid < 64) sh.T[0][lane] = 0.0f;
    __syncthreads();
    u32x4 wa[PW], wb[PW];
    load_split<G, W, PW>(rows + (size_t)q * ld, ((n + 3) & ~3) * 4, 0, ld, np, wv, lane, wa, wb);
    const int j = pick_split<G, W, PW>(wa, wb, n, np, wv, lane_bits, vis, sh.T[0], sh.w[0],
                                       us[q], lane);
    if (tid == 0) out[q] = j;
}

// Calls f.template operator()<G, W, PW>() for tile G, W waves and the pass
// count of n (PW = passes per wave).
template <typename F>
hipError_t dispatch_split(int tile, int waves, int n, F&& f) {
    const int passes = (n + 64 * tile - 1) / (64 * tile);
    if (tile == 8 && waves == 2 && passes == 2) return f.template operator()<8, 2, 1>();
    if (tile == 4 && waves == 2 && passes == 2) return f.template operator()<4, 2, 1>();
    if (tile == 4 && waves == 2 && (passes == 3 || passes == 4))
        return f.template operator()<4, 2, 2>();
    if (tile == 4 && waves == 4 && passes == 4) return f.template operator()<4, 4, 1>();
    return hipErrorInvalidValue;
}

}  // namespace

bool split_supported(int tile, int waves, int n) {
    if (n < 1 || n > kMaxSplitCities) return false;
    return dispatch_split(tile, waves, n, []<int G, int W, int PW>() { return hipSuccess; }) ==
           hipSuccess;
}

int construct_split_occupancy(const Colony& c) {
    int blocks = -1;
    (void)dispatch_split(c.tile, c.waves, c.n, [&]<int G, int W, int PW>() {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_construct_split<G, W, PW>,
                                                         64 * W, tour_lds_bytes(c.n)) !=
            hipSuccess)
            blocks = -1;
        return hipSuccess;
    });
    return blocks;
}

hipError_t launch_construct_split(const Colony& c, uint32_t iter, hipStream_t s) {
    return dispatch_split(c.tile, c.waves, c.n, [&]<int G, int W, int PW>() {
        hipLaunchKernelGGL((k_construct_split<G, W, PW>), dim3(c.m), dim3(64 * W),
                           tour_lds_bytes(c.n), s, c, iter);
        return hipGetLastError();
    });
}

hipError_t launch_test_select_split(int tile, int waves, int n, int count, const float* rows,
                                    const uint8_t* feasible, const float* u, int32_t* out,
                                    hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int ld = (n + 63) & ~63;
    return dispatch_split(tile, waves, n, [&]<int G, int W, int PW>() {
        hipLaunchKernelGGL((k_test_select_split<G, W, PW>), dim3(count), dim3(64 * W), 0, s,
                           rows, ld, n, feasible, u, out);
        return hipGetLastError();
    });
}

}  // namespace aco
