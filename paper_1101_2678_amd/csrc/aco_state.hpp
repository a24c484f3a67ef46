// aco_state.hpp -- device-side view of one colony and the launchers of the
// libaco kernels.  Host code only ever passes this struct by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace aco {

// One colony's arrays, carved out of the caller's workspace.
//   ld  row pitch (elements) of tau, choice, dist, delta: n rounded up to 64
//   tp  row pitch of tours: n+1 rounded up to 64
//   mp  row pitch of succ/pred: m rounded up to 64
struct Colony {
    int32_t n, m, ld, tp, mp;
    int32_t alpha, beta;
    float rho;
    uint64_t seed;
    float* tau;          // n x ld, FP32 pheromone; padding columns stay 0
    float* choice;       // n x ld, FP32 tau^alpha * eta^beta; padding 0
    int32_t* dist;       // n x ld, int32 distances; padding 0
    uint16_t* tours;     // m x tp, tour k in row k (n+1 entries)
    uint16_t* succ;      // n x mp: succ[i][k] = city after i in tour k
    uint16_t* pred;      // n x mp: pred[i][k] = city before i in tour k
    int64_t* lens;       // m tour lengths C^k
    float* dep;          // m deposits fl32(1 / C^k)
    int64_t* best_len;   // best-so-far length
    uint16_t* best_tour; // tp entries
    int64_t* cnn;        // nearest-neighbour tour length
    float* tau0;         // m / C_nn
    double* delta;       // n x ld binary64 deposits (atomic update), or null
    uint32_t* iter_dev;  // next iteration (batched path; advanced on the device)
    int32_t tile;        // construction tile: cities per lane per pass (4 or 8)
    int32_t waves;       // construction wavefronts per ant (1, or 2 / 4 for n <= 1024)
    int32_t dep_emin;    // every deposit fl32(1/C^k) has a binary32 exponent field >= this
};

constexpr int kMaxCities = 4096;
constexpr int kMaxTile4Cities = 1024;  // tile 4 holds 16 passes of 256 cities at most
// Largest n aco_update_atomic_noalloc takes (its static deposit matrix holds
// n * ld binary64 cells, ld = n rounded up to 64).
constexpr int kMaxNoallocCities = 1024;

// Whether the construction kernel has a variant with `tile` cities per lane
// for n cities.
bool tile_supported(int tile, int n);
hipError_t launch_construct(const Colony& c, uint32_t iter, hipStream_t s);
// Several wavefronts per ant (c.waves > 1): rows of at most kMaxSplitCities
// cities, W = 2 or 4 waves sharing the passes of tile c.tile, W <= passes.
constexpr int kMaxSplitCities = 1024;
bool split_supported(int tile, int waves, int n);
hipError_t launch_construct_split(const Colony& c, uint32_t iter, hipStream_t s);
int construct_split_occupancy(const Colony& c);
hipError_t launch_test_select_split(int tile, int waves, int n, int count, const float* rows,
                                    const uint8_t* feasible, const float* u, int32_t* out,
                                    hipStream_t s);
// One workgroup per entry of antmap: (colony << 16) | ant.  max_n, the largest
// n among the colonies, picks the kernel's pass bound, so it must not be
// smaller than any colony's n; lds (dynamic LDS per workgroup, from
// batch_lds_bytes) holds the tour and sets how many workgroups fit a CU.
hipError_t launch_construct_batch(const Colony* cols, const uint32_t* antmap, int total_ants,
                                  int max_n, size_t lds, hipStream_t s);
// Dynamic LDS per batched construction workgroup for at most wg_per_cu
// workgroups on a CU of lds_per_cu bytes (wg_per_cu 0: no cap, the tour only).
size_t batch_lds_bytes(int max_n, int wg_per_cu, size_t lds_per_cu);
// The cap a batch of total_ants ants on `cus` compute units gets by default.
int batch_default_cap(int total_ants, int cus);
hipError_t launch_best_batch(const Colony* cols, int count, hipStream_t s);
// One workgroup per entry of rowmap: (colony << 16) | row.
hipError_t launch_update_gather_batch(const Colony* cols, const uint32_t* rowmap, int total_rows,
                                      int max_ld, hipStream_t s);
// Construction workgroups (ants) resident per compute unit, or -1.
int construct_occupancy(const Colony& c);
hipError_t launch_update_gather(const Colony& c, hipStream_t s);
// combine_in_lds: the shared-memory deposit (one global atomic per distinct
// edge of a row's workgroup); false: one global atomic per tour edge.
hipError_t launch_update_atomic(const Colony& c, bool combine_in_lds, hipStream_t s);
hipError_t launch_init(const Colony& c, hipStream_t s);
hipError_t launch_refresh_choice(const Colony& c, hipStream_t s);
hipError_t launch_test_select(int tile, int n, int count, const float* rows,
                              const uint8_t* feasible, const float* u, int32_t* out,
                              hipStream_t s);
hipError_t launch_probe_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_probe_rows(const float* mat, int rows, int ld, int row_len, int waves,
                             int steps, int rows_in_flight, float* sink, hipStream_t s);
// loads: 16-byte loads in flight per thread (4, 8 or 16); nontemporal loads
// keep nothing in the caches.
hipError_t launch_probe_read(const void* src, size_t bytes, int reps, int loads, bool nontemporal,
                             float* sink, hipStream_t s);

}  // namespace aco
