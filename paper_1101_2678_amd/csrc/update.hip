// update.hip -- pheromone update (Section II, Eqs. 2-4; GPU designs in
// Section III-B), initialisation and the best-so-far tour.
//
// Both update variants produce the same bits: the deposits reaching a cell
// are binary32 values summed in binary64, and with at most m <= 2^16 terms
// whose exponents span at most 12 binades (every tour length lies between
// about 2 d_max and n d_max, n <= 4096) the sum needs fewer than 53 bits, so
// it is exact in any order.  The evaporated value and that sum are then
// added with a single rounding:  tau' = fl32((double)fl32(tau * keep) + D).
// The same bound makes the sum exact in fixed point: scaled by 2^S, with S
// such that the smallest deposit the instance can have is an integer, every
// deposit is an integer and every sum an integer below 2^53, so the LDS
// accumulators hold unsigned 64-bit integers (integer atomics, faster than
// binary64 ones on this part) and convert back to the same binary64 value
// exactly.
//
//   gather  (scatter-to-gather, Section III-B, without the O(n^4) scan): one
//           workgroup owns row i, reads succ[i][*] and pred[i][*] (the two
//           tour neighbours of city i in every ant's tour), accumulates the
//           deposits in 64-bit fixed-point LDS slots, then evaporates, adds and
//           refreshes the choice row.  No global atomics.
//   atomic  (Section III-B, "atomic instructions + shared memory", the
//           paper's fastest update): one thread per city of an ant's tour.
//           The threads of city i (the tours' edges leaving i, read from
//           succ[i][*]) first add their deposits in fixed-point LDS slots
//           keyed by the edge's other end; each non-zero slot then goes to the
//           upper-triangle cell of its undirected edge with one global
//           binary64 atomic, which merges the two directions an edge can be
//           travelled in.  An epilogue over pairs of 64 x 64 tiles
//           evaporates, adds the sum to both (i, j) and (j, i), refreshes the
//           choice matrix and clears the deposits.
//   atomic_direct (the paper's "atomic instructions" version): the same
//           epilogue, but every tour edge issues its own global atomic, with
//           no on-chip combining.
#include "aco_device.hpp"
#include "aco_state.hpp"
#include "nn.hpp"

namespace aco {
namespace {

constexpr int kRowThreads = 256;

// Fixed-point deposits.  c.dep_emin bounds the binary32 exponent field of
// every deposit from below (from the instance's longest possible tour) and
// fixes the scale 2^S, S = 150 - dep_emin: a deposit with exponent field e
// and 24-bit significand M is M << (e - dep_emin), exactly, and a sum A
// stands for A * 2^-S.  The bound on the tour lengths' spread that makes
// binary64 sums exact keeps every sum of up to m deposits below 2^53, so A
// converts back to binary64 exactly.
__device__ __forceinline__ unsigned long long fixed_of(float d, int e_min) {
    const uint32_t b = __float_as_uint(d);
    const uint32_t sig = (b & 0x7FFFFFu) | 0x800000u;  // deposits are normal, > 0
    return (unsigned long long)sig << (int)(((b >> 23) & 0xFFu) - (uint32_t)e_min);
}

__device__ __forceinline__ double value_of(unsigned long long a, int e_min) {
    return ldexp((double)a, e_min - 150);
}

__device__ __forceinline__ float evaporation_keep(float rho) {
    return (float)(1.0 - (double)rho);  // fl32(1 - rho)
}

__device__ __forceinline__ void apply_cell(float& tau, float& choice, int32_t d, double dsum,
                                           float keep, int alpha, int beta) {
    const float evaporated = tau * keep;
    tau = (float)((double)evaporated + dsum);
    choice = choice_of(tau, heur_of(d, beta), alpha);
}

__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
    return a < b ? a : b;
}

__device__ __forceinline__ unsigned long long wave_min64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = umin64(v, __shfl_xor(v, off));
    return v;
}

// ---------------------------------------------------------------------------
// Best-so-far: the shortest tour of this iteration (lowest ant index among
// equals) replaces the stored one only if strictly shorter.
// ---------------------------------------------------------------------------
// NT threads, every one of the workgroup.
template <int NT>
__device__ __forceinline__ void best_of(const Colony& c, bool advance_iter) {
    static_assert(NT % 64 == 0 && NT <= 1024, "whole wavefronts, at most 16");
    __shared__ unsigned long long part[NT / 64];
    __shared__ unsigned long long s_win;
    const int tid = threadIdx.x;
    unsigned long long best = ~0ull;
    for (int k = tid; k < c.m; k += NT)
        best = umin64(best, ((unsigned long long)c.lens[k] << 16) | (unsigned)k);
    best = wave_min64(best);
    if ((tid & 63) == 0) part[tid >> 6] = best;
    __syncthreads();
    if (tid < 64) {
        unsigned long long v = (tid < NT / 64) ? part[tid] : ~0ull;
        v = wave_min64(v);
        if (tid == 0) s_win = v;
    }
    __syncthreads();
    const long long len = (long long)(s_win >> 16);
    const int k = (int)(s_win & 0xffffu);
    const long long prev = *c.best_len;
    if (len < prev) {
        const uint16_t* src = c.tours + (size_t)k * c.tp;
        for (int s = tid; s <= c.n; s += NT) c.best_tour[s] = src[s];
        __syncthreads();
        if (tid == 0) *c.best_len = len;
    }
    // The batched path keeps each colony's iteration counter on the device,
    // so that a captured sequence of launches advances when replayed.
    if (advance_iter && tid == 0) *c.iter_dev += 1u;
}

// The deposits of row i (four ants at a time: one 8-byte load of four
// successors, one of four predecessors, one 16-byte load of four deposits)
// into the fixed-point LDS accumulators s_A.  With HOT, deposits to columns
// h0 and h1 are summed in registers and added once per wavefront: once the
// colony converges most ants share city i's two neighbours, and with many
// ants their deposits would queue on those two LDS slots.  Any h0, h1 give
// the same integer sums.
template <int T, bool HOT>
__device__ __forceinline__ void deposit_row(const Colony& c, int i, unsigned long long* s_A) {
    const int tid = threadIdx.x;
    const int e_min = c.dep_emin;
    const uint16_t* sr = c.succ + (size_t)i * c.mp;
    const uint16_t* pr = c.pred + (size_t)i * c.mp;
    const int m4 = c.m / 4;
    // ant 0's neighbours of city i: a guess of the two shared ones
    const uint32_t h0 = HOT ? sr[0] : 0u, h1 = HOT ? pr[0] : 0u;
    unsigned long long a0 = 0ull, a1 = 0ull;
    auto add = [&](uint32_t j, unsigned long long v) {
        if (HOT && j == h0)
            a0 += v;
        else if (HOT && j == h1)
            a1 += v;
        else
            atomicAdd(&s_A[j], v);
    };
    for (int q = tid; q < m4; q += T) {
        const ushort4 su = reinterpret_cast<const ushort4*>(sr)[q];
        const ushort4 pu = reinterpret_cast<const ushort4*>(pr)[q];
        const float4 dv = reinterpret_cast<const float4*>(c.dep)[q];
        const unsigned long long a = fixed_of(dv.x, e_min), b = fixed_of(dv.y, e_min);
        const unsigned long long g = fixed_of(dv.z, e_min), h = fixed_of(dv.w, e_min);
        add(su.x, a);
        add(pu.x, a);
        add(su.y, b);
        add(pu.y, b);
        add(su.z, g);
        add(pu.z, g);
        add(su.w, h);
        add(pu.w, h);
    }
    for (int k = 4 * m4 + tid; k < c.m; k += T) {
        const unsigned long long a = fixed_of(c.dep[k], e_min);
        add(sr[k], a);
        add(pr[k], a);
    }
    if (HOT) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off);
            a1 += __shfl_xor(a1, off);
        }
        if ((tid & 63) == 0) {
            if (a0) atomicAdd(&s_A[h0], a0);
            if (a1) atomicAdd(&s_A[h1], a1);
        }
    }
}

// Ants from which the gather update sums the likely shared neighbours in
// registers: n = m = 2400, 0.0293 -> 0.0265 ms (0.032 -> 0.028 ms once
// converged); at n = m = 1000 the extra compares cost more (0.0112 -> 0.0118).
constexpr int kHotAnts = 2048;

// Row i of the gather update by a workgroup of T threads: deposits into
// fixed-point LDS accumulators, cleared 16 bytes at a time, then evaporation,
// the deposits and the choice row.
template <int T>
__device__ __forceinline__ void gather_row(const Colony& c, int i, unsigned long long* s_A) {
    const int tid = threadIdx.x;
    ulonglong2* s_A2 = reinterpret_cast<ulonglong2*>(s_A);
    for (int j = tid; j < c.ld / 2; j += T) s_A2[j] = make_ulonglong2(0ull, 0ull);
    __syncthreads();
    if (c.m >= kHotAnts)
        deposit_row<T, true>(c, i, s_A);
    else
        deposit_row<T, false>(c, i, s_A);
    const int e_min = c.dep_emin;
    __syncthreads();
    const float keep = evaporation_keep(c.rho);
    float4* trow = reinterpret_cast<float4*>(c.tau + (size_t)i * c.ld);
    float4* crow = reinterpret_cast<float4*>(c.choice + (size_t)i * c.ld);
    const int4* drow = reinterpret_cast<const int4*>(c.dist + (size_t)i * c.ld);
    for (int q = tid; q < c.ld / 4; q += T) {
        float4 t = trow[q];
        const int4 d = drow[q];
        float4 ch;
        apply_cell(t.x, ch.x, d.x, value_of(s_A[4 * q + 0], e_min), keep, c.alpha, c.beta);
        apply_cell(t.y, ch.y, d.y, value_of(s_A[4 * q + 1], e_min), keep, c.alpha, c.beta);
        apply_cell(t.z, ch.z, d.z, value_of(s_A[4 * q + 2], e_min), keep, c.alpha, c.beta);
        apply_cell(t.w, ch.w, d.w, value_of(s_A[4 * q + 3], e_min), keep, c.alpha, c.beta);
        trow[q] = t;
        crow[q] = ch;
    }
}

// Threads per row of the single-instance gather update.  Each row's
// accumulators take ld 64-bit words of LDS, which caps the rows a compute
// unit holds (8 at n = 2400, 2048 on the device for 2400 rows); more threads
// per row shorten each row, so the rows that do not fit the first round cost
// less.
constexpr int kGatherThreads = 256;

// Workgroup 0 also keeps the best-so-far tour (it reads only the lengths and
// tours of the construction, which the update does not touch), so one launch
// serves both.
__global__ __launch_bounds__(kGatherThreads) void k_update_gather(Colony c) {
    extern __shared__ __align__(16) unsigned long long s_A[];  // ld accumulators
    if (blockIdx.x == 0) best_of<kGatherThreads>(c, false);
    gather_row<kGatherThreads>(c, blockIdx.x, s_A);
}

// Batched gather: workgroup g updates row (rowmap[g] & 0xffff) of colony
// cols[rowmap[g] >> 16].
__global__ __launch_bounds__(kRowThreads) void k_update_gather_batch(
    const Colony* __restrict__ cols, const uint32_t* __restrict__ rowmap) {
    extern __shared__ __align__(16) unsigned long long s_A[];
    const uint32_t e = rowmap[blockIdx.x];
    const Colony c = cols[e >> 16];
    gather_row<kRowThreads>(c, (int)(e & 0xffffu), s_A);
}

// grid (ceil(n / 256), m): thread (s, k) adds ant k's deposit for the tour
// edge {tour_k[s], tour_k[s+1]}.  On a symmetric instance (i, j) and (j, i)
// receive the same sum, so one binary64 atomic into the upper-triangle cell
// delta[min][max] stands for both; the epilogue reads it for both cells.
__global__ __launch_bounds__(256) void k_deposit_atomic(Colony c) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y;
    if (s >= c.n) return;
    const uint16_t* t = c.tours + (size_t)k * c.tp;
    const int i = t[s], j = t[s + 1];
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    unsafeAtomicAdd(&c.delta[(size_t)lo * c.ld + hi], (double)c.dep[k]);
}

// grid (n, slices): workgroup (i, q) takes the ants k = q, q + slices, ...
// (interleaved, so every slice reads whole contiguous runs of succ[i][*]).
// Thread t adds dep_k for the edge i -> succ_k(i) into fixed-point LDS slot
// succ_k(i); the non-zero slots then go out, converted back to binary64
// (exactly), as one global atomic each.  An ant's tour holds an undirected
// edge at most once, so each deposit reaches its cell exactly once, and the
// sums stay exact whatever the grouping.
__global__ __launch_bounds__(kRowThreads) void k_deposit_shared(Colony c) {
    extern __shared__ __align__(16) unsigned long long s_A[];  // one slot per other end j
    const int i = blockIdx.x;
    const int tid = threadIdx.x;
    for (int j = tid; j < c.ld; j += kRowThreads) s_A[j] = 0ull;
    __syncthreads();
    const int e_min = c.dep_emin;
    const uint16_t* sr = c.succ + (size_t)i * c.mp;
    const int step = (int)gridDim.y * kRowThreads;
    if (c.m >= kHotAnts) {
        // as in deposit_row: ant 0's two neighbours of i summed in registers
        const uint32_t h0 = sr[0], h1 = c.pred[(size_t)i * c.mp];
        unsigned long long a0 = 0ull, a1 = 0ull;
        for (int k = (int)blockIdx.y * kRowThreads + tid; k < c.m; k += step) {
            const uint32_t j = sr[k];
            const unsigned long long v = fixed_of(c.dep[k], e_min);
            if (j == h0)
                a0 += v;
            else if (j == h1)
                a1 += v;
            else
                atomicAdd(&s_A[j], v);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off);
            a1 += __shfl_xor(a1, off);
        }
        if ((tid & 63) == 0) {
            if (a0) atomicAdd(&s_A[h0], a0);
            if (a1) atomicAdd(&s_A[h1], a1);
        }
    } else {
        for (int k = (int)blockIdx.y * kRowThreads + tid; k < c.m; k += step)
            atomicAdd(&s_A[sr[k]], fixed_of(c.dep[k], e_min));
    }
    __syncthreads();
    for (int j = tid; j < c.n; j += kRowThreads) {
        const unsigned long long a = s_A[j];
        if (a != 0ull) {
            const int lo = i < j ? i : j, hi = i < j ? j : i;
            unsafeAtomicAdd(&c.delta[(size_t)lo * c.ld + hi], value_of(a, e_min));
        }
    }
}

// Ant slices of the shared-memory deposit: enough workgroups to fill the
// device (about 2048) when there are few rows, never fewer than 256 ants a
// slice.
int deposit_slices(int n, int m) {
    const int by_ants = (m + kRowThreads - 1) / kRowThreads;
    const int by_rows = (2048 + n - 1) / n;
    const int s = by_rows < by_ants ? by_rows : by_ants;
    return s < 1 ? 1 : s;
}

constexpr int kTile = 64;

// Tile pair (I, J) = (blockIdx.y, blockIdx.x), I <= J, of 64 x 64 cells
// (grid ld/64 x ld/64; pairs with I > J exit at once).  The upper-triangle
// deposits of tile (I, J) are staged in LDS (rows beyond n as zeros); tau and
// choice of tile (I, J) take them as they are, those of tile (J, I) take them
// transposed (in a diagonal tile the lower cells read the upper ones), so
// every cell gets the sum of its undirected edge; then the staged cells are
// cleared.  Every global access is a contiguous row segment.
__global__ __launch_bounds__(256) void k_update_epilogue(Colony c) {
    __shared__ double s_d[kTile][kTile + 1];
    const int I = blockIdx.y, J = blockIdx.x;
    if (I > J) return;
    if (I == 0 && J == 0) best_of<256>(c, false);  // as in k_update_gather
    const int tid = threadIdx.x;
    const int rr = tid / 16, c0 = (tid % 16) * 4;  // rows rr + 16 q, columns c0 .. c0 + 3
    const float keep = evaporation_keep(c.rho);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = rr + 16 * q, i = I * kTile + r;
        double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
        if (i < c.n) {
            const double2* dp =
                reinterpret_cast<const double2*>(c.delta + (size_t)i * c.ld + J * kTile + c0);
            a = dp[0];
            b = dp[1];
        }
        s_d[r][c0 + 0] = a.x;
        s_d[r][c0 + 1] = a.y;
        s_d[r][c0 + 2] = b.x;
        s_d[r][c0 + 3] = b.y;
    }
    __syncthreads();
    // tile (I, J)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = rr + 16 * q, i = I * kTile + r;
        if (i >= c.n) continue;
        const size_t off = (size_t)i * c.ld + J * kTile + c0;
        float4 t = *reinterpret_cast<float4*>(c.tau + off);
        const int4 d = *reinterpret_cast<const int4*>(c.dist + off);
        double D[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int col = c0 + e;
            D[e] = (I < J || r <= col) ? s_d[r][col] : s_d[col][r];
        }
        float4 ch;
        apply_cell(t.x, ch.x, d.x, D[0], keep, c.alpha, c.beta);
        apply_cell(t.y, ch.y, d.y, D[1], keep, c.alpha, c.beta);
        apply_cell(t.z, ch.z, d.z, D[2], keep, c.alpha, c.beta);
        apply_cell(t.w, ch.w, d.w, D[3], keep, c.alpha, c.beta);
        *reinterpret_cast<float4*>(c.tau + off) = t;
        *reinterpret_cast<float4*>(c.choice + off) = ch;
    }
    // tile (J, I): cell (J*64 + r, I*64 + col) is the upper cell (I*64 + col, J*64 + r)
    if (I < J) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rr + 16 * q, i = J * kTile + r;
            if (i >= c.n) continue;
            const size_t off = (size_t)i * c.ld + I * kTile + c0;
            float4 t = *reinterpret_cast<float4*>(c.tau + off);
            const int4 d = *reinterpret_cast<const int4*>(c.dist + off);
            float4 ch;
            apply_cell(t.x, ch.x, d.x, s_d[c0 + 0][r], keep, c.alpha, c.beta);
            apply_cell(t.y, ch.y, d.y, s_d[c0 + 1][r], keep, c.alpha, c.beta);
            apply_cell(t.z, ch.z, d.z, s_d[c0 + 2][r], keep, c.alpha, c.beta);
            apply_cell(t.w, ch.w, d.w, s_d[c0 + 3][r], keep, c.alpha, c.beta);
            *reinterpret_cast<float4*>(c.tau + off) = t;
            *reinterpret_cast<float4*>(c.choice + off) = ch;
        }
    }
    // clear the staged upper-triangle cells
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = I * kTile + rr + 16 * q;
        if (i >= c.n) continue;
        double2* dp = reinterpret_cast<double2*>(c.delta + (size_t)i * c.ld + J * kTile + c0);
        dp[0] = make_double2(0.0, 0.0);
        dp[1] = make_double2(0.0, 0.0);
    }
}

// ---------------------------------------------------------------------------
// Initialisation: C_nn by the nearest-neighbour tour from city 0 (ties to the
// lowest index) and tau0 = fl32(m / C_nn) come from launch_nn_tour
// (construct_nn.hip); the fill below sets tau and choice.
// ---------------------------------------------------------------------------
// grid (ceil(ld / 4 / 256), n): tau <- tau0 (padding 0), choice from tau,
// delta <- 0 when present.
__global__ __launch_bounds__(256) void k_fill_init(Colony c) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int i = blockIdx.y;
    if (q >= c.ld / 4) return;
    const size_t off = (size_t)i * c.ld + 4 * (size_t)q;
    const float t0 = *c.tau0;
    const int4 d = *reinterpret_cast<const int4*>(c.dist + off);
    const int j = 4 * q;
    float4 t, ch;
    t.x = (j + 0 < c.n) ? t0 : 0.0f;
    t.y = (j + 1 < c.n) ? t0 : 0.0f;
    t.z = (j + 2 < c.n) ? t0 : 0.0f;
    t.w = (j + 3 < c.n) ? t0 : 0.0f;
    ch.x = choice_of(t.x, heur_of(d.x, c.beta), c.alpha);
    ch.y = choice_of(t.y, heur_of(d.y, c.beta), c.alpha);
    ch.z = choice_of(t.z, heur_of(d.z, c.beta), c.alpha);
    ch.w = choice_of(t.w, heur_of(d.w, c.beta), c.alpha);
    *reinterpret_cast<float4*>(c.tau + off) = t;
    *reinterpret_cast<float4*>(c.choice + off) = ch;
    if (c.delta) {
        double2* dp = reinterpret_cast<double2*>(c.delta + off);
        dp[0] = make_double2(0.0, 0.0);
        dp[1] = make_double2(0.0, 0.0);
    }
}

// grid (ceil(ld / 4 / 256), n): choice from the current tau (checkpoint restore).
__global__ __launch_bounds__(256) void k_refresh_choice(Colony c) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int i = blockIdx.y;
    if (q >= c.ld / 4) return;
    const size_t off = (size_t)i * c.ld + 4 * (size_t)q;
    const float4 t = *reinterpret_cast<const float4*>(c.tau + off);
    const int4 d = *reinterpret_cast<const int4*>(c.dist + off);
    float4 ch;
    ch.x = choice_of(t.x, heur_of(d.x, c.beta), c.alpha);
    ch.y = choice_of(t.y, heur_of(d.y, c.beta), c.alpha);
    ch.z = choice_of(t.z, heur_of(d.z, c.beta), c.alpha);
    ch.w = choice_of(t.w, heur_of(d.w, c.beta), c.alpha);
    *reinterpret_cast<float4*>(c.choice + off) = ch;
}

__global__ __launch_bounds__(1024) void k_best_batch(const Colony* __restrict__ cols) {
    const Colony c = cols[blockIdx.x];
    best_of<1024>(c, true);
}

dim3 cell_grid(const Colony& c) { return dim3((c.ld / 4 + 255) / 256, c.n); }

}  // namespace

hipError_t launch_update_gather(const Colony& c, hipStream_t s) {
    hipLaunchKernelGGL(k_update_gather, dim3(c.n), dim3(kGatherThreads),
                       (size_t)c.ld * sizeof(unsigned long long), s, c);
    return hipGetLastError();
}

hipError_t launch_update_atomic(const Colony& c, bool combine_in_lds, hipStream_t s) {
    if (!c.delta) return hipErrorInvalidValue;
    if (combine_in_lds)
        hipLaunchKernelGGL(k_deposit_shared, dim3(c.n, deposit_slices(c.n, c.m)),
                           dim3(kRowThreads), (size_t)c.ld * sizeof(unsigned long long), s, c);
    else
        hipLaunchKernelGGL(k_deposit_atomic, dim3((c.n + 255) / 256, c.m), dim3(256), 0, s, c);
    const int nt = c.ld / kTile;
    hipLaunchKernelGGL(k_update_epilogue, dim3(nt, nt), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_init(const Colony& c, hipStream_t s) {
    const hipError_t e = launch_nn_tour(c, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_init, cell_grid(c), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_refresh_choice(const Colony& c, hipStream_t s) {
    hipLaunchKernelGGL(k_refresh_choice, cell_grid(c), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_best_batch(const Colony* cols, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_best_batch, dim3(count), dim3(1024), 0, s, cols);
    return hipGetLastError();
}

hipError_t launch_update_gather_batch(const Colony* cols, const uint32_t* rowmap, int total_rows,
                                      int max_ld, hipStream_t s) {
    if (total_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_gather_batch, dim3(total_rows), dim3(kRowThreads),
                       (size_t)max_ld * sizeof(unsigned long long), s, cols, rowmap);
    return hipGetLastError();
}

}  // namespace aco
