// noalloc.hip -- the atomic pheromone update (Section II, Eqs. 2-4; the
// atomic design of Section III-B) with its binary64 deposit matrix held in a
// library-owned static device array instead of the caller's workspace, for
// callers that cannot allocate device memory.
//
// `scratch` is one array per GPU, alive until the process ends.  Host code
// never uses its name as an address: the address each device gives it is
// looked up once per device (hipGetSymbolAddress, with that device current,
// from aco_init) and kept in a table; kernels and the clearing launch take
// that address.  Every call on one GPU shares the array: it is cleared at
// the start of each call, and calls that overlap on one GPU (contexts on
// different streams) race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "aco.h"
#include "aco_ctx.hpp"
#include "aco_host.hpp"
#include "aco_state.hpp"

namespace aco {
namespace {

// n * ld binary64 cells at most: n <= 1024 (ld = 1024), 8 MiB per GPU.
constexpr size_t kScratchDoubles = (size_t)kMaxNoallocCities * kMaxNoallocCities;

static __device__ __align__(256) double scratch[kScratchDoubles];

// Clears `count` doubles (a multiple of 2) at p with 16-byte stores.  A
// kernel rather than hipMemsetAsync, so a captured sequence replays it as
// plain work.
__global__ __launch_bounds__(256) void k_zero_f64(double2* __restrict__ p, size_t count2) {
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count2; i += stride)
        p[i] = make_double2(0.0, 0.0);
}

constexpr int kMaxDevices = 64;

struct ScratchSlot {
    bool looked_up;
    hipError_t err;
    void* ptr;
};

std::mutex g_scratch_mu;
ScratchSlot g_scratch[kMaxDevices];

}  // namespace

namespace host {

hipError_t noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchSlot& s = g_scratch[device];
    if (!s.looked_up) {
        void* p = nullptr;
        s.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        // a failed lookup must not surface later as some launch's error
        if (s.err != hipSuccess) (void)hipGetLastError();
        s.ptr = s.err == hipSuccess ? p : nullptr;
        s.looked_up = true;
    }
    *out = s.ptr;
    return s.err;
}

}  // namespace host
}  // namespace aco

extern "C" aco_status aco_update_atomic_noalloc(aco_ctx* c) {
    using aco::host::fail;
    if (aco_status s = aco::host::update_ready(c)) return s;
    const size_t cells = (size_t)c->col.n * (size_t)c->col.ld;
    if (cells > aco::kScratchDoubles)
        return fail(ACO_ERR_INVALID,
                    "aco_update_atomic_noalloc: n = " + std::to_string(c->col.n) +
                        " is above the static deposit matrix's limit of n <= " +
                        std::to_string(aco::kMaxNoallocCities));
    if (!c->scratch)
        return fail(ACO_ERR_DEVICE,
                    std::string("aco_update_atomic_noalloc: no device address for the static "
                                "deposit matrix (") +
                        hipGetErrorString(c->scratch_err) + ")");
    const size_t count2 = cells / 2;  // ld is a multiple of 64
    const int blocks = (int)((count2 + 255) / 256 < 1024 ? (count2 + 255) / 256 : 1024);
    hipLaunchKernelGGL(aco::k_zero_f64, dim3(blocks), dim3(256), 0, c->stream,
                       static_cast<double2*>(c->scratch), count2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return aco::host::device_fail(&c->poisoned, e, "aco_update_atomic_noalloc");
    return aco::host::enqueue_update(c, ACO_UPDATE_ATOMIC, static_cast<double*>(c->scratch));
}
