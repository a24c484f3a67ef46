// aco_ctx.hpp -- the host-side state behind an aco_ctx handle, shared by the
// translation units that implement the single-instance entry points.
#pragma once

#include <hip/hip_runtime.h>

#include "aco.h"
#include "aco_state.hpp"
#include "nn.hpp"

struct aco_ctx {
    aco::Colony col;
    aco::NnTables nn;       // candidate lists; nn.nn == 0 until aco_nn_attach
    hipStream_t stream;
    int device;             // the HIP device current at aco_init
    size_t ws_bytes;
    uint32_t next_iter;     // first iteration aco_solve runs
    uint32_t pending_iter;  // iteration of the construction awaiting update
    bool pending;           // a construction has not been followed by an update
    bool poisoned;
    bool has_atomic;
    void* scratch;          // this device's address of the static deposit matrix, or null
    hipError_t scratch_err; // why it is null
};

namespace aco {
namespace host {

// Enqueues the update of `kind` on the context's stream after the call-order
// checks of aco_update.  `delta` replaces the workspace's binary64 deposit
// matrix for the atomic kind (nullptr: the workspace's own).
aco_status enqueue_update(aco_ctx* c, aco_update_kind kind, double* delta);
// ACO_OK if the context can take an update now (not poisoned, a
// construction pending), else the status aco_update would return.
aco_status update_ready(aco_ctx* c);
// Device address of the static deposit matrix of aco_update_atomic_noalloc
// on `device`, which must be current; looked up on the first call for each
// device and remembered.  *out is null if the lookup failed.
hipError_t noalloc_scratch(int device, void** out);

}  // namespace host
}  // namespace aco
