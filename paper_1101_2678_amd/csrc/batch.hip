// batch.hip -- many independent Ant System instances advanced together, and
// the construction-tile autotuner.
//
// A batch keeps every instance resident in one caller-owned workspace.  One
// AS iteration of the whole batch is three launches: construction of every
// ant of every instance (one workgroup per ant, instances ordered largest n
// first so the longest tours start first), the best-so-far of every
// instance, and the gather update of every row of every instance.  Each
// instance keeps its own iteration counter on the device, so the launches of
// `iters` iterations can be captured once into a HIP graph and replayed.
// Every instance computes exactly what it computes alone (same kernels' code,
// same Philox keys), whatever the batch around it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <unordered_set>
#include <vector>

#include "aco.h"
#include "aco_host.hpp"
#include "aco_state.hpp"

using aco::host::fail;

struct aco_batch {
    int32_t count = 0;
    std::vector<aco::Colony> cols;     // caller order
    std::vector<int> order;            // launch position -> caller index
    aco::Colony* d_cols = nullptr;     // launch order
    uint32_t* d_antmap = nullptr;      // (position << 16) | ant
    uint32_t* d_rowmap = nullptr;      // (position << 16) | row
    int total_ants = 0, total_rows = 0, max_n = 0, max_ld = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t graph_iters = 0;
    bool poisoned = false;
    // launch configuration of the construction (speed only, never results)
    aco_batch_config config{0, -1};
    int cus = 0;                   // compute units of the device
    size_t lds_per_cu = 0;         // LDS bytes per compute unit
    size_t max_lds_per_wg = 0;     // LDS bytes one workgroup may hold
    std::vector<aco::Colony> launch_cols;  // host copy of d_cols
};

namespace {

struct BatchLayout {
    std::vector<size_t> inst_off;
    std::vector<aco::host::Layout> inst;
    size_t cols_off = 0, antmap_off = 0, rowmap_off = 0, end = 0;
    int total_ants = 0, total_rows = 0;
};

bool batch_layout(int32_t count, const aco_params* params, BatchLayout* B, std::string* why) {
    if (count < 1 || count > 65535) return (*why = "count must be in [1, 65535]", false);
    if (!params) return (*why = "params is NULL", false);
    size_t off = 0;
    B->inst_off.resize(count);
    B->inst.resize(count);
    for (int q = 0; q < count; ++q) {
        if (!aco::host::params_valid(&params[q], why)) {
            *why = "instance " + std::to_string(q) + ": " + *why;
            return false;
        }
        B->inst[q] = aco::host::make_layout(params[q]);
        B->inst_off[q] = off;
        off += aco::host::round_up(B->inst[q].base_end, aco::host::kAlign);
        B->total_ants += params[q].m;
        B->total_rows += params[q].n;
    }
    B->cols_off = off;
    off += aco::host::round_up((size_t)count * sizeof(aco::Colony), aco::host::kAlign);
    B->antmap_off = off;
    off += aco::host::round_up((size_t)B->total_ants * sizeof(uint32_t), aco::host::kAlign);
    B->rowmap_off = off;
    off += aco::host::round_up((size_t)B->total_rows * sizeof(uint32_t), aco::host::kAlign);
    B->end = off;
    return true;
}

aco_status batch_usable(aco_batch* b) {
    if (!b) return fail(ACO_ERR_INVALID, "batch is NULL");
    if (b->poisoned) return fail(ACO_ERR_STATE, "batch poisoned by an earlier device error");
    return ACO_OK;
}

aco_status batch_device_fail(aco_batch* b, hipError_t e, const char* where) {
    return aco::host::device_fail(b ? &b->poisoned : nullptr, e, where);
}

hipError_t enqueue_iterations(aco_batch* b, uint32_t iters) {
    hipError_t e = hipSuccess;
    for (uint32_t i = 0; i < iters && e == hipSuccess; ++i) {
        e = aco::launch_construct_batch(
            b->d_cols, b->d_antmap, b->total_ants, b->max_n,
            aco::batch_lds_bytes(b->max_n, b->config.wg_per_cu, b->lds_per_cu), b->stream);
        if (e == hipSuccess) e = aco::launch_best_batch(b->d_cols, b->count, b->stream);
        if (e == hipSuccess)
            e = aco::launch_update_gather_batch(b->d_cols, b->d_rowmap, b->total_rows, b->max_ld,
                                                b->stream);
    }
    return e;
}

// Waits for the batch's stream (a replay of the graph may still be running)
// before releasing the graph.
void drop_graph(aco_batch* b) {
    if (b->exec || b->graph) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_iters = 0;
}

// ---- synthetic instance for the autotuner: distinct points uniform in
// [0, 10^6]^2 from a 64-bit xorshift stream, nint Euclidean distances.
struct Xorshift {
    uint64_t s;
    uint64_t next() {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        return s;
    }
};

std::vector<int32_t> tuning_instance(int n) {
    Xorshift g{0x9E3779B97F4A7C15ull ^ (uint64_t)n};
    std::vector<int64_t> x, y;
    std::unordered_set<uint64_t> seen;
    while ((int)x.size() < n) {
        const int64_t px = (int64_t)(g.next() % 1000001ull), py = (int64_t)(g.next() % 1000001ull);
        if (seen.insert(((uint64_t)px << 32) | (uint64_t)py).second) {
            x.push_back(px);
            y.push_back(py);
        }
    }
    std::vector<int32_t> d((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const double dx = (double)(x[i] - x[j]), dy = (double)(y[i] - y[j]);
            d[(size_t)i * n + j] = (int32_t)std::floor(std::sqrt(dx * dx + dy * dy) + 0.5);
        }
    return d;
}

}  // namespace

extern "C" {

size_t aco_batch_workspace_bytes(int32_t count, const aco_params* params) {
    BatchLayout B;
    std::string why;
    if (!batch_layout(count, params, &B, &why)) return 0;
    return B.end;
}

aco_status aco_batch_init(aco_batch** out, int32_t count, const aco_params* params,
                          const int32_t* const* dist_hosts, void* d_workspace, size_t ws_bytes,
                          void* hip_stream) {
    aco::host::g_error.clear();
    if (!out) return fail(ACO_ERR_INVALID, "out is NULL");
    *out = nullptr;
    BatchLayout B;
    std::string why;
    if (!batch_layout(count, params, &B, &why)) return fail(ACO_ERR_INVALID, why);
    if (!dist_hosts) return fail(ACO_ERR_INVALID, "dist_hosts is NULL");
    std::vector<int> dep_emin(count, 0);
    for (int q = 0; q < count; ++q) {
        if (!dist_hosts[q]) return fail(ACO_ERR_INVALID, "dist_hosts[" + std::to_string(q) + "] is NULL");
        if (!aco::host::dist_valid(dist_hosts[q], params[q].n, params[q].m, &why, &dep_emin[q]))
            return fail(ACO_ERR_INVALID, "instance " + std::to_string(q) + ": " + why);
    }
    if (!d_workspace || ((uintptr_t)d_workspace % aco::host::kAlign) != 0)
        return fail(ACO_ERR_NOMEM, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < B.end) return fail(ACO_ERR_NOMEM, "workspace smaller than aco_batch_workspace_bytes");
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess)
        return fail(ACO_ERR_DEVICE, "aco_batch_init: no current HIP device");
    if (aco_status s = aco::host::stream_on_device(hip_stream, device, "aco_batch_init")) return s;

    int cus = 0, max_wg_lds = 0;
    size_t lds_per_cu = 0;
    if (aco::host::device_shape(&cus, &lds_per_cu) != hipSuccess ||
        hipDeviceGetAttribute(&max_wg_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
            hipSuccess)
        return fail(ACO_ERR_DEVICE, "aco_batch_init: device attributes unavailable");
    aco_batch* b = new (std::nothrow) aco_batch();
    if (!b) return fail(ACO_ERR_NOMEM, "host allocation failed");
    b->cus = cus;
    b->lds_per_cu = lds_per_cu;
    b->max_lds_per_wg = (size_t)max_wg_lds;
    b->config.wg_per_cu = aco::batch_default_cap(B.total_ants, cus);
    b->config.tile4_max_n = -1;
    char* base = static_cast<char*>(d_workspace);
    b->count = count;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->cols.resize(count);
    hipError_t e = hipSuccess;
    for (int q = 0; q < count && e == hipSuccess; ++q) {
        b->cols[q] = aco::host::carve(base + B.inst_off[q], B.inst[q], params[q], false,
                                      dep_emin[q], aco::host::tile_for(params[q].n));
        e = aco::host::upload_and_init(b->cols[q], dist_hosts[q], B.inst[q].base_end, b->stream);
        b->max_n = std::max(b->max_n, params[q].n);
        b->max_ld = std::max(b->max_ld, B.inst[q].ld);
    }
    b->order.resize(count);
    for (int q = 0; q < count; ++q) b->order[q] = q;
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int a, int c) { return params[a].n > params[c].n; });
    std::vector<aco::Colony>& launch_cols = b->launch_cols;
    launch_cols.resize(count);
    std::vector<uint32_t> antmap, rowmap;
    antmap.reserve(B.total_ants);
    rowmap.reserve(B.total_rows);
    for (int pos = 0; pos < count; ++pos) {
        const int q = b->order[pos];
        launch_cols[pos] = b->cols[q];
        for (int k = 0; k < params[q].m; ++k) antmap.push_back(((uint32_t)pos << 16) | (uint32_t)k);
        for (int i = 0; i < params[q].n; ++i) rowmap.push_back(((uint32_t)pos << 16) | (uint32_t)i);
    }
    b->total_ants = B.total_ants;
    b->total_rows = B.total_rows;
    b->d_cols = reinterpret_cast<aco::Colony*>(base + B.cols_off);
    b->d_antmap = reinterpret_cast<uint32_t*>(base + B.antmap_off);
    b->d_rowmap = reinterpret_cast<uint32_t*>(base + B.rowmap_off);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_cols, launch_cols.data(), sizeof(aco::Colony) * count,
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_antmap, antmap.data(), sizeof(uint32_t) * antmap.size(),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_rowmap, rowmap.data(), sizeof(uint32_t) * rowmap.size(),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        const aco_status s = batch_device_fail(b, e, "aco_batch_init");
        delete b;
        return s;
    }
    *out = b;
    return ACO_OK;
}

aco_status aco_batch_run(aco_batch* b, uint32_t iters, int32_t use_graph) {
    if (aco_status s = batch_usable(b)) return s;
    if (iters == 0) return ACO_OK;
    hipError_t e;
    if (!use_graph) {
        e = enqueue_iterations(b, iters);
        if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_run");
        return ACO_OK;
    }
    if (!b->stream)
        return fail(ACO_ERR_INVALID, "graph capture needs a non-default stream");
    if (!b->exec || b->graph_iters != iters) {
        drop_graph(b);
        e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_run: begin capture");
        const hipError_t enq = enqueue_iterations(b, iters);
        e = hipStreamEndCapture(b->stream, &b->graph);
        if (enq != hipSuccess) e = enq;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return batch_device_fail(b, e, "aco_batch_run: capture");
        }
        b->graph_iters = iters;
    }
    e = hipGraphLaunch(b->exec, b->stream);
    if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_run: graph launch");
    return ACO_OK;
}

aco_status aco_batch_sync(aco_batch* b) {
    if (aco_status s = batch_usable(b)) return s;
    const hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_sync");
    return ACO_OK;
}

static aco_status batch_instance(aco_batch* b, int32_t q, const aco::Colony** col) {
    if (aco_status s = batch_usable(b)) return s;
    if (q < 0 || q >= b->count) return fail(ACO_ERR_INVALID, "instance index out of range");
    if (aco_status s = aco_batch_sync(b)) return s;
    *col = &b->cols[q];
    return ACO_OK;
}

aco_status aco_batch_read_best(aco_batch* b, int32_t q, uint16_t* best_tour_host,
                               int64_t* best_len_host) {
    const aco::Colony* c;
    if (aco_status s = batch_instance(b, q, &c)) return s;
    hipError_t e = hipSuccess;
    if (best_len_host) e = hipMemcpy(best_len_host, c->best_len, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && best_tour_host)
        e = hipMemcpy(best_tour_host, c->best_tour, ((size_t)c->n + 1) * sizeof(uint16_t),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_read_best");
    return ACO_OK;
}

aco_status aco_batch_read_tours(aco_batch* b, int32_t q, uint16_t* tours_host, int64_t* lens_host) {
    const aco::Colony* c;
    if (aco_status s = batch_instance(b, q, &c)) return s;
    hipError_t e = hipSuccess;
    if (tours_host)
        e = hipMemcpy2D(tours_host, ((size_t)c->n + 1) * sizeof(uint16_t), c->tours,
                        (size_t)c->tp * sizeof(uint16_t), ((size_t)c->n + 1) * sizeof(uint16_t),
                        (size_t)c->m, hipMemcpyDeviceToHost);
    if (e == hipSuccess && lens_host)
        e = hipMemcpy(lens_host, c->lens, (size_t)c->m * sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_read_tours");
    return ACO_OK;
}

aco_status aco_batch_read_tau(aco_batch* b, int32_t q, float* tau_host) {
    const aco::Colony* c;
    if (aco_status s = batch_instance(b, q, &c)) return s;
    if (!tau_host) return fail(ACO_ERR_INVALID, "tau_host is NULL");
    const hipError_t e =
        hipMemcpy2D(tau_host, (size_t)c->n * sizeof(float), c->tau, (size_t)c->ld * sizeof(float),
                    (size_t)c->n * sizeof(float), (size_t)c->n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_read_tau");
    return ACO_OK;
}

aco_status aco_batch_get_iter(aco_batch* b, int32_t q, uint32_t* iter) {
    const aco::Colony* c;
    if (aco_status s = batch_instance(b, q, &c)) return s;
    if (!iter) return fail(ACO_ERR_INVALID, "iter is NULL");
    const hipError_t e = hipMemcpy(iter, c->iter_dev, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_get_iter");
    return ACO_OK;
}

void aco_batch_destroy(aco_batch* b) {
    if (!b) return;
    drop_graph(b);
    delete b;
}

aco_status aco_batch_set_config(aco_batch* b, const aco_batch_config* cfg) {
    if (aco_status s = batch_usable(b)) return s;
    if (!cfg) return fail(ACO_ERR_INVALID, "config is NULL");
    if (cfg->wg_per_cu < 0 || cfg->wg_per_cu > 64)
        return fail(ACO_ERR_INVALID, "wg_per_cu must be in [0, 64]");
    if (aco::batch_lds_bytes(b->max_n, cfg->wg_per_cu, b->lds_per_cu) > b->max_lds_per_wg)
        return fail(ACO_ERR_INVALID, "wg_per_cu asks for more LDS than one workgroup may hold");
    if (cfg->tile4_max_n < -1 || cfg->tile4_max_n > aco::kMaxTile4Cities)
        return fail(ACO_ERR_INVALID, "tile4_max_n must be in [-1, 1024]");
    // the graph holds the old launch shape; a replay still queued reads d_cols
    drop_graph(b);
    hipError_t e = hipStreamSynchronize(b->stream);
    for (int pos = 0; pos < b->count; ++pos) {
        const int q = b->order[pos];
        const int n = b->cols[q].n;
        const int tile = cfg->tile4_max_n < 0 ? aco::host::tile_for(n)
                                              : (n <= cfg->tile4_max_n ? 4 : 8);
        b->cols[q].tile = tile;
        b->launch_cols[pos].tile = tile;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_cols, b->launch_cols.data(), sizeof(aco::Colony) * b->count,
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_set_config");
    b->config = *cfg;
    return ACO_OK;
}

aco_status aco_batch_get_config(aco_batch* b, aco_batch_config* cfg) {
    if (aco_status s = batch_usable(b)) return s;
    if (!cfg) return fail(ACO_ERR_INVALID, "config is NULL");
    *cfg = b->config;
    return ACO_OK;
}

aco_status aco_batch_autotune(aco_batch* b, const aco_batch_config* cands, int32_t count,
                              uint32_t iters, int32_t* best_index, float* ms_per_iter) {
    if (aco_status s = batch_usable(b)) return s;
    if (!cands || count < 1) return fail(ACO_ERR_INVALID, "need at least one candidate");
    if (iters < 1) return fail(ACO_ERR_INVALID, "iters must be >= 1");
    for (int i = 0; i < count; ++i) {
        if (cands[i].wg_per_cu < 0 || cands[i].wg_per_cu > 64 ||
            aco::batch_lds_bytes(b->max_n, cands[i].wg_per_cu, b->lds_per_cu) > b->max_lds_per_wg ||
            cands[i].tile4_max_n < -1 || cands[i].tile4_max_n > aco::kMaxTile4Cities)
            return fail(ACO_ERR_INVALID, "candidate " + std::to_string(i) + " is out of range");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best = 0;
    float t_best = 1e30f;
    for (int i = 0; i < count && e == hipSuccess; ++i) {
        if (aco_status s = aco_batch_set_config(b, &cands[i])) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return s;
        }
        e = enqueue_iterations(b, 1);  // warm-up at this shape
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess) e = enqueue_iterations(b, iters);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        ms /= (float)iters;
        if (ms_per_iter) ms_per_iter[i] = ms;
        if (ms < t_best) {
            t_best = ms;
            best = i;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return batch_device_fail(b, e, "aco_batch_autotune");
    if (best_index) *best_index = best;
    return aco_batch_set_config(b, &cands[best]);
}

aco_status aco_autotune(void* d_workspace, size_t ws_bytes, const int32_t* sizes, int32_t count,
                        int32_t reps, void* hip_stream, int32_t* chosen_tile,
                        int32_t* chosen_waves, float* ms) {
    // The shapes timed, in the order of ms's columns (aco.h).
    constexpr int kShapes[ACO_NUM_SHAPES][2] = {{4, 1}, {8, 1}, {8, 2}, {4, 2}, {4, 4}};
    aco::host::g_error.clear();
    if (!sizes || count < 1) return fail(ACO_ERR_INVALID, "need at least one size");
    if (reps < 1) return fail(ACO_ERR_INVALID, "reps must be >= 1");
    for (int i = 0; i < count; ++i) {
        if (sizes[i] < 3 || sizes[i] > aco::kMaxCities)
            return fail(ACO_ERR_INVALID, "sizes must be in [3, 4096]");
        if (i > 0 && sizes[i] <= sizes[i - 1])
            return fail(ACO_ERR_INVALID, "sizes must be strictly increasing");
    }
    const aco_params pmax{sizes[count - 1], sizes[count - 1], 1, 2, 0.5f, 1};
    const aco::host::Layout Lmax = aco::host::make_layout(pmax);
    if (!d_workspace || ((uintptr_t)d_workspace % aco::host::kAlign) != 0)
        return fail(ACO_ERR_NOMEM, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < Lmax.base_end)
        return fail(ACO_ERR_NOMEM, "workspace smaller than aco_workspace_bytes(largest size, m = n)");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    std::vector<int> best(count, 1);  // index into kShapes
    for (int i = 0; i < count && e == hipSuccess; ++i) {
        const int n = sizes[i];
        const aco_params p{n, n, 1, 2, 0.5f, 1};
        const aco::host::Layout L = aco::host::make_layout(p);
        const std::vector<int32_t> d = tuning_instance(n);
        // construction only: the deposits' scale is not used, but is filled in
        std::string why;
        int dep_emin = 0;
        (void)aco::host::dist_valid(d.data(), n, n, &why, &dep_emin);
        float t_best = 1e30f;
        for (int k = 0; k < ACO_NUM_SHAPES; ++k) {
            const int tile = kShapes[k][0], waves = kShapes[k][1];
            if (ms) ms[(size_t)i * ACO_NUM_SHAPES + k] = -1.0f;
            if (!aco::host::shape_supported(tile, waves, n)) continue;
            const aco::Colony col =
                aco::host::carve(static_cast<char*>(d_workspace), L, p, false, dep_emin, tile,
                                 waves);
            e = aco::host::upload_and_init(col, d.data(), L.base_end, s);
            if (e == hipSuccess) e = aco::launch_construct(col, 0, s);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = aco::launch_construct(col, (uint32_t)r + 1u, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) break;
            t /= (float)reps;
            if (ms) ms[(size_t)i * ACO_NUM_SHAPES + k] = t;
            if (t < t_best) {
                t_best = t;
                best[i] = k;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return aco::host::device_fail(nullptr, e, "aco_autotune");
    // Size bucket i covers (sizes[i-1], sizes[i]]; the last bucket runs to
    // 4096.  A size of the bucket that the chosen shape does not support takes
    // the chosen tile with one wavefront, or tile 8 where tile 4 stops.
    for (int i = 0; i < count; ++i) {
        const int lo = i == 0 ? 1 : sizes[i - 1] + 1;
        const int hi = i == count - 1 ? aco::kMaxCities : sizes[i];
        const int tile = kShapes[best[i]][0], waves = kShapes[best[i]][1];
        for (int n = lo; n <= hi; ++n) {
            if (aco::host::shape_supported(tile, waves, n))
                aco::host::set_shape_range(n, n, tile, waves);
            else if (aco::tile_supported(tile, n))
                aco::host::set_shape_range(n, n, tile, 1);
            else
                aco::host::set_shape_range(n, n, 8, 1);
        }
        if (chosen_tile) chosen_tile[i] = tile;
        if (chosen_waves) chosen_waves[i] = waves;
    }
    return ACO_OK;
}

}  // extern "C"
