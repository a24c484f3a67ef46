// construct_nn.hip -- tour construction over nearest-neighbour candidate
// lists (Section II, the candidate-list variant of Eq. (1); the paper's GPU
// versions 4-6 of Table II).
//
// At city i the candidates are the entries of i's list (the nn nearest
// cities, ordered by (d_ij, j)).  If any of them is unvisited, the next city
// is drawn by the R64 roulette over the list in list order: lane r holds
// candidate r with weight choice[i][nnl[i][r]] if it is unvisited, else +0;
// one S64 prefix over the 64 lanes gives the prefixes, and the pick is the
// lowest unvisited r whose prefix exceeds fl32(u * total), else the highest
// unvisited r.  With a single 64-entry block the block offset is +0, so this
// is the full-row rule applied to the candidate vector.  If every candidate
// is visited, the next city is the unvisited city of largest choice value
// (lowest index among equal values), found by one pass over the row.
//
// One wavefront per ant.  Per step the wave reads one packed row of the
// candidate table (8 bytes per candidate, in L2 for every instance size the
// library accepts), so the kernel is bound by the latency of that dependent
// load and of the selection that follows it, not by bandwidth; the rare
// fallback issues all loads of the 4n-byte choice row at once.  The kernel
// is specialised on the number of 256-city passes of the fallback and on
// whether the list fits the low 32 lanes.
#include <hip/hip_runtime.h>

#include "aco_device.hpp"
#include "aco_state.hpp"
#include "nn.hpp"

namespace aco {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

size_t round_up256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t tour_bytes(int n) { return ((size_t)(n + 1) * sizeof(uint16_t) + 15) & ~(size_t)15; }

// LDS of one ant: a visited flag per city (1 = visited, or >= n), then the
// tour.  Byte flags make a visit one plain byte store and let the fallback
// read the flags of four consecutive cities with one 32-bit load.
constexpr size_t kVisBytes = kMaxCities;

size_t construct_nn_lds(int n) { return kVisBytes + tour_bytes(n); }

// S64 restricted to lanes 0..31 (stage A and the row_bcast:15 step).  When
// lanes 32..63 hold +0, lanes 0..31 of the full tree end with these values
// and its last lane with the value of lane 31: row 3 adds (+0 + +0) + X
// with X = fl(R1 + R0), the value lane 31 gets here.
__device__ __forceinline__ float s64_scan_lo32(float x) {
    x = x + dpp_move<0x111, 0xF>(x);
    x = x + dpp_move<0x112, 0xF>(x);
    x = x + dpp_move<0x114, 0xF>(x);
    x = x + dpp_move<0x118, 0xF>(x);
    x = x + dpp_move<0x142, 0xA>(x);
    return x;
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, kCtrl, kRowMask, 0xF, false);
}

// Wave maximum / minimum through the same DPP tree (lanes with no source
// take the neutral element); the result is read from lane 63, so it is
// wave-uniform.
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

// The unvisited city with the largest choice value, lowest index among equal
// values, for a row of n <= 256 P cities.  Choice values are finite and
// >= +0, so their bit patterns order like the values; key = bits + 1 (0 for
// "none").  Lane l holds cities 256 p + 4 l .. +3 of every pass p: all P
// loads are issued before any is used (loads past the row, rounded up to 4
// cities, return 0, and those cities are flagged visited).  Each lane keeps
// its first maximum in increasing city order; the wave takes the largest
// key, then the lowest city among the lanes holding it.
template <int P>
__device__ __forceinline__ int fallback_argmax(const float* row, int n, const uint8_t* vis,
                                               int lane) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(row), (short)0, ((n + 3) & ~3) * 4, 0x00020000);
    u32x4 q[P];
#pragma unroll
    for (int p = 0; p < P; ++p)
        q[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, (256 * p + 4 * lane) * 4, 0, 0);
    uint32_t flags[P];
#pragma unroll
    for (int p = 0; p < P; ++p) flags[p] = reinterpret_cast<const uint32_t*>(vis)[64 * p + lane];
    // keep every load above in flight before the first use below (one memory
    // round trip instead of one per few passes)
    __builtin_amdgcn_sched_barrier(0);
    uint32_t best = 0;
    uint32_t best_j = ~0u;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t key = q[p][e] + 1u;
            if (((flags[p] >> (8 * e)) & 0xFFu) == 0u && key > best) {
                best = key;
                best_j = (uint32_t)(256 * p + 4 * lane + e);
            }
        }
    const uint32_t top = wave_max_u32(best);
    const uint32_t j = wave_min_u32(best == top && best != 0u ? best_j : ~0u);
    return top == 0u ? -1 : (int)j;
}

// Packed candidate table from the current choice matrix.
__global__ __launch_bounds__(256) void k_cand_refresh(Colony c, NnTables t) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= c.n * t.kp) return;
    const int i = idx / t.kp, r = idx - i * t.kp;
    uint64_t v = 0;
    if (r < t.nn) {
        const int j = t.nnl[idx];
        v = ((uint64_t)j << 32) | __float_as_uint(c.choice[(size_t)i * c.ld + j]);
    }
    t.cand[idx] = v;
}

// Row i's list: nn rounds of a workgroup minimum over the keys
// (d_ij << 32) | j, each round taking the smallest key above the previous
// one.  Keys are distinct (j is), so the rounds enumerate the row in
// (d_ij, j) order; j = i and padding get the key 2^64 - 1 and are never
// taken because nn <= n - 1.
__global__ __launch_bounds__(256) void k_nn_lists(Colony c, NnTables t) {
    __shared__ uint64_t part[4];
    const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = c.n;
    uint64_t key[kMaxCities / 256];
#pragma unroll
    for (int q = 0; q < kMaxCities / 256; ++q) {
        const int j = tid + 256 * q;
        key[q] = (j < n && j != i)
                     ? ((uint64_t)(uint32_t)c.dist[(size_t)i * c.ld + j] << 32) | (uint64_t)j
                     : ~0ull;
    }
    uint16_t* out = t.nnl + (size_t)i * t.kp;
    uint64_t prev = 0;
    for (int r = 0; r < t.nn; ++r) {
        uint64_t mn = ~0ull;
#pragma unroll
        for (int q = 0; q < kMaxCities / 256; ++q)
            if (key[q] > prev && key[q] < mn) mn = key[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor((unsigned long long)mn, off);
            mn = o < mn ? o : mn;
        }
        if (lane == 0) part[wave] = mn;
        __syncthreads();
        mn = part[0];
#pragma unroll
        for (int w = 1; w < 4; ++w) mn = part[w] < mn ? part[w] : mn;
        __syncthreads();
        if (tid == 0) out[r] = (uint16_t)(mn & 0xFFFFu);
        prev = mn;
    }
    for (int r = t.nn + tid; r < t.kp; r += 256) out[r] = 0;
}

template <int P, bool kNn32>
__global__ __launch_bounds__(64) void k_construct_nn(Colony c, NnTables t, uint32_t iter) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint8_t* s_vis = smem;
    uint16_t* s_tour = reinterpret_cast<uint16_t*>(smem + kVisBytes);
    const int lane = threadIdx.x;
    const int k = ant_of_block(blockIdx.x, c.m);
    const int n = c.n, nn = t.nn, kp = t.kp;
    const PhiloxKey key{(uint32_t)c.seed, (uint32_t)(c.seed >> 32)};

    for (int w = lane; w < (int)(kVisBytes / 4); w += 64) {
        uint32_t f = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) f |= (4 * w + b >= n ? 1u : 0u) << (8 * b);
        reinterpret_cast<uint32_t*>(s_vis)[w] = f;
    }
    __syncthreads();

    const uint32_t x0 = draw(key, iter, (uint32_t)k, 0u);
    int cur = (int)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);

    // Lanes kp..63 re-read entries of the same row (kp is 32 or 64), so the
    // load needs no branch; only lanes < nn can be candidates.
    const int col = lane & (kp - 1);
    const bool in_list = lane < nn;
    const uint64_t list_mask = nn == 64 ? ~0ull : (1ull << nn) - 1ull;
    // the row offset goes in the scalar offset, so no vector address math sits
    // between the selected city and the next load (every access is in range)
    const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
        t.cand, (short)0, n * kp * (int)sizeof(uint64_t), 0x00020000);
    // A step's candidate row is loaded as soon as its city is known; the
    // city's bookkeeping (tour entry, visited flag) follows the load, before
    // the flags are read (one wavefront: its LDS accesses stay in order).
    float u64 = 0.0f;
    for (int step = 1; step < n; ++step) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(
            crs, col * (int)sizeof(uint64_t), cur * kp * (int)sizeof(uint64_t), 0);
        if (lane == 0) {
            s_tour[step - 1] = (uint16_t)cur;
            s_vis[cur] = 1;
        }
        const int slot = (step - 1) & 63;
        if (__builtin_expect(slot == 0, 0))
            u64 = uniform24(draw(key, iter, (uint32_t)k, (uint32_t)(step + lane)));
        const float u = read_lane(u64, slot);

        const int city = (int)v.y;
        // every lane reads its flag (a valid index on every lane), so the
        // read needs no branch; `&` keeps it unconditional
        const bool unvisited = s_vis[city] == 0;
        const bool feas = in_list & unvisited;
        const float w = feas ? __uint_as_float(v.x) : 0.0f;
        const float s = kNn32 ? s64_scan_lo32(w) : s64_scan(w);
        const float target = u * read_lane(s, kNn32 ? 31 : 63);
        const uint64_t live = ballot(unvisited) & list_mask;
        int next;
        if (__builtin_expect(live != 0, 1)) {
            const uint64_t hit = ballot(s > target) & live;
            const int r = hit ? __builtin_ctzll(hit) : 63 - __builtin_clzll(live);
            next = __builtin_amdgcn_readlane(city, r);
        } else {
            next = fallback_argmax<P>(c.choice + (size_t)cur * c.ld, n, s_vis, lane);
            // n - step >= 1 cities are unvisited, so next >= 0; the clamp only
            // keeps the LDS indices in range should that ever break.
            next = next < 0 ? 0 : next;
        }
        cur = next;
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

// Launches k_construct_nn<P, nn <= 32> for P = ceil(n / 256) in 1..16.
template <int P>
hipError_t launch_nn_passes(const Colony& c, const NnTables& t, uint32_t iter, hipStream_t s) {
    if constexpr (P > kMaxCities / 256) {
        return hipErrorInvalidValue;
    } else {
        if ((c.n + 255) / 256 != P) return launch_nn_passes<P + 1>(c, t, iter, s);
        const size_t lds = construct_nn_lds(c.n);
        if (t.nn <= 32)
            hipLaunchKernelGGL((k_construct_nn<P, true>), dim3(c.m), dim3(64), lds, s, c, t, iter);
        else
            hipLaunchKernelGGL((k_construct_nn<P, false>), dim3(c.m), dim3(64), lds, s, c, t,
                               iter);
        return hipGetLastError();
    }
}

// The unseen city nearest to the row's city (smallest d, lowest index among
// equal d), for a row of n <= 256 P cities: all P 16-byte loads are issued
// before any is used; loads past the row (rounded up to 4 cities) return 0,
// and those cities are flagged seen.  -1 if every city is seen.
template <int P>
__device__ __forceinline__ int nearest_unseen(const int32_t* row, int n, const uint8_t* seen,
                                              int lane) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t*>(row), (short)0, ((n + 3) & ~3) * 4, 0x00020000);
    u32x4 q[P];
#pragma unroll
    for (int p = 0; p < P; ++p)
        q[p] = __builtin_amdgcn_raw_buffer_load_b128(rs, (256 * p + 4 * lane) * 4, 0, 0);
    uint32_t flags[P];
#pragma unroll
    for (int p = 0; p < P; ++p) flags[p] = reinterpret_cast<const uint32_t*>(seen)[64 * p + lane];
    __builtin_amdgcn_sched_barrier(0);
    uint32_t best = ~0u, best_j = ~0u;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // distances are >= 1 and < 2^31, so ~0 never stands for a city
            const uint32_t d = ((flags[p] >> (8 * e)) & 0xFFu) ? ~0u : q[p][e];
            if (d < best) {
                best = d;
                best_j = (uint32_t)(256 * p + 4 * lane + e);
            }
        }
    const uint32_t top = wave_min_u32(best);
    const uint32_t j = wave_min_u32(best == top ? best_j : ~0u);
    return top == ~0u ? -1 : (int)j;
}

// C_nn, the length of the nearest-neighbour tour from city 0 (ties to the
// lowest index), and tau0 = fl32(m / C_nn).  Row i of the (d, j)-sorted lists
// holds i's nearest cities, so its first unseen entry is the nearest unseen
// city overall (every city off the list has a larger (d, j) key); only when
// every entry is seen does the wave scan the whole distance row.  One
// wavefront; the tour is kept in LDS and summed at the end.
template <int P>
__global__ __launch_bounds__(64) void k_nn_tour_lists(Colony c, NnTables t) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint8_t* s_seen = smem;
    uint16_t* s_tour = reinterpret_cast<uint16_t*>(smem + kVisBytes);
    const int lane = threadIdx.x;
    const int n = c.n, nn = t.nn, kp = t.kp;
    for (int w = lane; w < (int)(kVisBytes / 4); w += 64) {
        uint32_t f = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) f |= (4 * w + b >= n || 4 * w + b == 0 ? 1u : 0u) << (8 * b);
        reinterpret_cast<uint32_t*>(s_seen)[w] = f;
    }
    if (lane == 0) s_tour[0] = 0;
    __syncthreads();
    const int col = lane & (kp - 1);
    const bool in_list = lane < nn;
    int cur = 0;
    for (int step = 1; step < n; ++step) {
        const int city = t.nnl[(size_t)cur * kp + col];
        const bool unseen = in_list & (s_seen[city] == 0);
        const uint64_t live = ballot(unseen);
        int next;
        if (live) {
            next = __builtin_amdgcn_readlane(city, __builtin_ctzll(live));
        } else {
            next = nearest_unseen<P>(c.dist + (size_t)cur * c.ld, n, s_seen, lane);
            // n - step >= 1 cities are unseen, so next >= 0; the clamp only
            // keeps the LDS indices in range should that ever break.
            next = next < 0 ? 0 : next;
        }
        if (lane == 0) {
            s_tour[step] = (uint16_t)next;
            s_seen[next] = 1;
        }
        cur = next;
    }
    __syncthreads();
    long long len = 0;
    for (int s = lane; s < n; s += 64) {
        const int i = s_tour[s], j = s + 1 < n ? s_tour[s + 1] : 0;
        len += c.dist[(size_t)i * c.ld + j];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) len += __shfl_xor(len, off);
    if (lane == 0) {
        *c.cnn = len;
        *c.tau0 = (float)((double)c.m / (double)len);
        *c.best_len = 0x7fffffffffffffffLL;
    }
}

template <int P>
hipError_t launch_nn_tour_passes(const Colony& c, const NnTables& t, hipStream_t s) {
    if constexpr (P > kMaxCities / 256) {
        return hipErrorInvalidValue;
    } else {
        if ((c.n + 255) / 256 != P) return launch_nn_tour_passes<P + 1>(c, t, s);
        hipLaunchKernelGGL((k_nn_tour_lists<P>), dim3(1), dim3(64), construct_nn_lds(c.n), s, c,
                           t);
        return hipGetLastError();
    }
}

}  // namespace

hipError_t launch_nn_tour(const Colony& c, hipStream_t s) {
    if (c.n < 2 || c.n > kMaxCities || c.mp < 32) return hipErrorInvalidValue;
    // The successor table (n x mp uint16, mp >= 64) is not used before the
    // first construction, so it holds the 32-entry lists meanwhile.
    NnTables t{};
    t.nn = c.n - 1 < 32 ? c.n - 1 : 32;
    t.kp = 32;
    t.nnl = c.succ;
    t.cand = nullptr;
    hipError_t e = launch_nn_lists(c, t, s);
    if (e != hipSuccess) return e;
    return launch_nn_tour_passes<1>(c, t, s);
}

size_t nn_table_bytes(int n, int nn) {
    const size_t kp = (size_t)nn_pitch(nn);
    return round_up256((size_t)n * kp * sizeof(uint16_t)) +
           round_up256((size_t)n * kp * sizeof(uint64_t));
}

NnTables nn_carve(char* base, int n, int nn) {
    NnTables t{};
    t.nn = nn;
    t.kp = nn_pitch(nn);
    t.nnl = reinterpret_cast<uint16_t*>(base);
    t.cand = reinterpret_cast<uint64_t*>(base +
                                         round_up256((size_t)n * t.kp * sizeof(uint16_t)));
    return t;
}

hipError_t launch_nn_lists(const Colony& c, const NnTables& t, hipStream_t s) {
    if (t.nn < 1 || t.nn > kMaxNn || t.nn > c.n - 1 || c.n > kMaxCities)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_nn_lists, dim3(c.n), dim3(256), 0, s, c, t);
    return hipGetLastError();
}

hipError_t launch_construct_nn(const Colony& c, const NnTables& t, uint32_t iter, hipStream_t s) {
    if (t.nn < 1 || t.nn > kMaxNn || t.nn > c.n - 1 || c.n > kMaxCities)
        return hipErrorInvalidValue;
    const int cells = c.n * t.kp;
    hipLaunchKernelGGL(k_cand_refresh, dim3((cells + 255) / 256), dim3(256), 0, s, c, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_nn_passes<1>(c, t, iter, s);
}

}  // namespace aco
