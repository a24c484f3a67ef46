// aco_host.hpp -- host-side helpers shared by the C ABI translation units
// (validation, workspace layout, colony carving, the construction tile table).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "aco.h"
#include "aco_state.hpp"

namespace aco {
namespace host {

constexpr size_t kAlign = 256;

// Byte offsets of every array of one colony inside its workspace.
struct Layout {
    int32_t ld, tp, mp;
    size_t tau, choice, dist, tours, succ, pred, lens, dep, best_len, best_tour, cnn, tau0, iter,
        delta, base_end, atomic_end;
};

extern thread_local std::string g_error;

aco_status fail(aco_status s, const std::string& why);
// Records a device failure (poisoning the owner if `poisoned` is given).
aco_status device_fail(bool* poisoned, hipError_t e, const char* where);
size_t round_up(size_t v, size_t a);
// ACO_OK if hip_stream (NULL: the default stream) is a stream of this HIP
// runtime on `device`; otherwise the failure is recorded under `where`.
aco_status stream_on_device(void* hip_stream, int device, const char* where);
bool params_valid(const aco_params* p, std::string* why);
// Checks the distances; dep_emin (may be NULL) receives a lower bound on the
// binary32 exponent field of every deposit fl32(1/C^k) the instance can have.
bool dist_valid(const int32_t* d, int n, int m, std::string* why, int* dep_emin = nullptr);
Layout make_layout(const aco_params& p);
Colony carve(char* base, const Layout& L, const aco_params& p, bool with_delta, int dep_emin,
             int tile, int waves = 1);
// Clears the colony's base arrays, uploads the distances and enqueues the
// initialisation kernels (nearest-neighbour tour, tau0, tau and choice fill).
hipError_t upload_and_init(const Colony& col, const int32_t* dist_host, size_t base_bytes,
                           hipStream_t stream);
// Compute units and LDS bytes per compute unit of the current device.
hipError_t device_shape(int* cus, size_t* lds_per_cu);
// Construction shape table: tile (cities per lane) and wavefronts per ant by n.
int tile_for(int n);
int waves_for(int n);
bool shape_supported(int tile, int waves, int n);
bool set_shape_range(int lo, int hi, int tile, int waves);
bool set_tile_range(int lo, int hi, int tile);
void reset_tiles();

}  // namespace host
}  // namespace aco
