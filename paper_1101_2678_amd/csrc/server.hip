// server.hip -- continuous batching of independent Ant System solves.
//
// A server owns a caller-provided device pool.  A request (an instance and a
// number of iterations) is admitted when a slot is free and the pool has a
// free block for the request's whole workspace (first fit; the footprint is
// aco_workspace_bytes without the atomic part).  Its distances are uploaded
// and its colony initialised on the server's admission stream; it joins the
// running set at the first tick after that work has finished.  A tick
// advances every running request by one AS iteration with the batched
// kernels (one construction launch over all their ants, one best-so-far
// launch, one gather launch over all their rows), so requests that arrive
// while others run share the device.  A request whose iterations are done
// leaves the set; its result stays readable until the slot is released.
// Every request computes exactly what a context of its own computes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "aco.h"
#include "aco_host.hpp"
#include "aco_state.hpp"

using aco::host::fail;

namespace {

enum SlotState : int { kFree = 0, kInit = 1, kRunning = 2, kDone = 3 };

struct Slot {
    SlotState state = kFree;
    aco::Colony col{};
    size_t off = 0, bytes = 0;
    uint32_t iters_total = 0, iters_queued = 0;
    int64_t request_id = -1;
    hipEvent_t ready = nullptr;  // initialisation finished
};

}  // namespace

struct aco_server {
    char* pool = nullptr;
    size_t pool_bytes = 0;
    std::map<size_t, size_t> free_blocks;  // offset -> size, coalesced
    std::vector<Slot> slots;
    // Device tables of the running set (in the pool's reserved head).
    aco::Colony* d_cols = nullptr;
    uint32_t* d_antmap = nullptr;
    uint32_t* d_rowmap = nullptr;
    int max_ants = 0, max_rows = 0;
    std::vector<int> running;  // slot indices in launch order (largest n first)
    int total_ants = 0, total_rows = 0, max_n = 0, max_ld = 0;
    bool dirty = false;
    hipStream_t stream = nullptr;      // ticks
    hipStream_t init_stream = nullptr; // admissions (library-owned)
    uint64_t ticks = 0;
    bool poisoned = false;
};

namespace {

aco_status server_usable(aco_server* s) {
    if (!s) return fail(ACO_ERR_INVALID, "server is NULL");
    if (s->poisoned) return fail(ACO_ERR_STATE, "server poisoned by an earlier device error");
    return ACO_OK;
}

aco_status server_fail(aco_server* s, hipError_t e, const char* where) {
    return aco::host::device_fail(s ? &s->poisoned : nullptr, e, where);
}

bool pool_alloc(aco_server* s, size_t bytes, size_t* off) {
    bytes = aco::host::round_up(bytes, aco::host::kAlign);
    for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t rest_off = it->first + bytes;
            s->free_blocks.erase(it);
            if (rest) s->free_blocks[rest_off] = rest;
            return true;
        }
    }
    return false;
}

void pool_free(aco_server* s, size_t off, size_t bytes) {
    bytes = aco::host::round_up(bytes, aco::host::kAlign);
    auto it = s->free_blocks.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != s->free_blocks.end() && it->first + it->second == next->first) {
        it->second += next->second;
        s->free_blocks.erase(next);
    }
    if (it != s->free_blocks.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            s->free_blocks.erase(it);
        }
    }
}

size_t largest_free(const aco_server* s) {
    size_t best = 0;
    for (const auto& kv : s->free_blocks) best = std::max(best, kv.second);
    return best;
}

// Moves finished initialisations into the running set and rebuilds the
// device tables if the set changed.  Called between ticks only.
hipError_t refresh_running(aco_server* s) {
    for (size_t i = 0; i < s->slots.size(); ++i) {
        Slot& sl = s->slots[i];
        if (sl.state != kInit) continue;
        const hipError_t q = hipEventQuery(sl.ready);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return q;
        sl.state = kRunning;
        s->dirty = true;
    }
    if (!s->dirty) return hipSuccess;
    std::vector<int> run;
    for (size_t i = 0; i < s->slots.size(); ++i)
        if (s->slots[i].state == kRunning && s->slots[i].iters_queued < s->slots[i].iters_total)
            run.push_back((int)i);
    std::stable_sort(run.begin(), run.end(),
                     [&](int a, int b) { return s->slots[a].col.n > s->slots[b].col.n; });
    std::vector<aco::Colony> cols;
    std::vector<uint32_t> antmap, rowmap;
    int max_n = 0, max_ld = 0;
    for (size_t pos = 0; pos < run.size(); ++pos) {
        const aco::Colony& c = s->slots[run[pos]].col;
        cols.push_back(c);
        for (int k = 0; k < c.m; ++k) antmap.push_back(((uint32_t)pos << 16) | (uint32_t)k);
        for (int r = 0; r < c.n; ++r) rowmap.push_back(((uint32_t)pos << 16) | (uint32_t)r);
        max_n = std::max(max_n, c.n);
        max_ld = std::max(max_ld, c.ld);
    }
    // The previous tick may still read the tables: wait for it first.
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess && !cols.empty())
        e = hipMemcpy(s->d_cols, cols.data(), sizeof(aco::Colony) * cols.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !antmap.empty())
        e = hipMemcpy(s->d_antmap, antmap.data(), sizeof(uint32_t) * antmap.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !rowmap.empty())
        e = hipMemcpy(s->d_rowmap, rowmap.data(), sizeof(uint32_t) * rowmap.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    s->running = run;
    s->total_ants = (int)antmap.size();
    s->total_rows = (int)rowmap.size();
    s->max_n = max_n;
    s->max_ld = max_ld;
    s->dirty = false;
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t aco_server_table_bytes(int32_t max_slots, int32_t max_ants, int32_t max_rows) {
    if (max_slots < 1 || max_slots > 65535 || max_ants < 1 || max_rows < 1) return 0;
    const size_t a = aco::host::kAlign;
    return aco::host::round_up((size_t)max_slots * sizeof(aco::Colony), a) +
           aco::host::round_up((size_t)max_ants * sizeof(uint32_t), a) +
           aco::host::round_up((size_t)max_rows * sizeof(uint32_t), a);
}

aco_status aco_server_create(aco_server** out, void* d_pool, size_t pool_bytes, int32_t max_slots,
                             int32_t max_ants, int32_t max_rows, void* hip_stream) {
    aco::host::g_error.clear();
    if (!out) return fail(ACO_ERR_INVALID, "out is NULL");
    *out = nullptr;
    const size_t head = aco_server_table_bytes(max_slots, max_ants, max_rows);
    if (head == 0) return fail(ACO_ERR_INVALID, "max_slots in [1, 65535], max_ants and max_rows >= 1");
    if (!d_pool || ((uintptr_t)d_pool % aco::host::kAlign) != 0)
        return fail(ACO_ERR_NOMEM, "pool must be a 256-byte aligned device pointer");
    if (pool_bytes < head) return fail(ACO_ERR_NOMEM, "pool smaller than aco_server_table_bytes");
    aco_server* s = new (std::nothrow) aco_server();
    if (!s) return fail(ACO_ERR_NOMEM, "host allocation failed");
    s->pool = static_cast<char*>(d_pool);
    s->pool_bytes = pool_bytes;
    s->slots.resize(max_slots);
    s->max_ants = max_ants;
    s->max_rows = max_rows;
    const size_t a = aco::host::kAlign;
    s->d_cols = reinterpret_cast<aco::Colony*>(s->pool);
    s->d_antmap = reinterpret_cast<uint32_t*>(
        s->pool + aco::host::round_up((size_t)max_slots * sizeof(aco::Colony), a));
    s->d_rowmap = reinterpret_cast<uint32_t*>(
        reinterpret_cast<char*>(s->d_antmap) +
        aco::host::round_up((size_t)max_ants * sizeof(uint32_t), a));
    if (pool_bytes > head) s->free_blocks[head] = pool_bytes - head;
    s->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipStreamCreateWithFlags(&s->init_stream, hipStreamNonBlocking);
    for (size_t i = 0; i < s->slots.size() && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&s->slots[i].ready, hipEventDisableTiming);
    if (e != hipSuccess) {
        const aco_status st = server_fail(s, e, "aco_server_create");
        aco_server_destroy(s);
        return st;
    }
    *out = s;
    return ACO_OK;
}

aco_status aco_server_submit(aco_server* s, const aco_params* p, const int32_t* dist_host,
                             uint32_t iters, int64_t request_id, int32_t* slot_out) {
    if (aco_status st = server_usable(s)) return st;
    if (!slot_out) return fail(ACO_ERR_INVALID, "slot_out is NULL");
    *slot_out = -1;
    std::string why;
    if (!aco::host::params_valid(p, &why)) return fail(ACO_ERR_INVALID, why);
    if (!dist_host) return fail(ACO_ERR_INVALID, "dist_host is NULL");
    if (iters < 1) return fail(ACO_ERR_INVALID, "iters must be >= 1");
    if (!aco::host::dist_valid(dist_host, p->n, p->m, &why)) return fail(ACO_ERR_INVALID, why);
    int free_slot = -1;
    int running_ants = 0, running_rows = 0;
    for (size_t i = 0; i < s->slots.size(); ++i) {
        const Slot& sl = s->slots[i];
        if (sl.state == kFree && free_slot < 0) free_slot = (int)i;
        if (sl.state == kInit || sl.state == kRunning) {
            running_ants += sl.col.m;
            running_rows += sl.col.n;
        }
    }
    if (free_slot < 0) return fail(ACO_ERR_STATE, "no free slot");
    if (running_ants + p->m > s->max_ants || running_rows + p->n > s->max_rows)
        return fail(ACO_ERR_STATE, "the running set would exceed max_ants or max_rows");
    const aco::host::Layout L = aco::host::make_layout(*p);
    size_t off = 0;
    if (!pool_alloc(s, L.base_end, &off)) return fail(ACO_ERR_NOMEM, "no free pool block large enough");
    Slot& sl = s->slots[free_slot];
    sl.col = aco::host::carve(s->pool + off, L, *p, false, aco::host::tile_for(p->n));
    sl.off = off;
    sl.bytes = L.base_end;
    sl.iters_total = iters;
    sl.iters_queued = 0;
    sl.request_id = request_id;
    hipError_t e = aco::host::upload_and_init(sl.col, dist_host, L.base_end, s->init_stream);
    if (e == hipSuccess) e = hipEventRecord(sl.ready, s->init_stream);
    if (e != hipSuccess) {
        pool_free(s, off, L.base_end);
        return server_fail(s, e, "aco_server_submit");
    }
    sl.state = kInit;
    *slot_out = free_slot;
    return ACO_OK;
}

aco_status aco_server_step(aco_server* s, int32_t* running_out) {
    if (aco_status st = server_usable(s)) return st;
    hipError_t e = refresh_running(s);
    if (e != hipSuccess) return server_fail(s, e, "aco_server_step");
    if (running_out) *running_out = (int32_t)s->running.size();
    if (s->running.empty()) return ACO_OK;
    e = aco::launch_construct_batch(s->d_cols, s->d_antmap, s->total_ants, s->max_n, s->stream);
    if (e == hipSuccess) e = aco::launch_best_batch(s->d_cols, (int)s->running.size(), s->stream);
    if (e == hipSuccess)
        e = aco::launch_update_gather_batch(s->d_cols, s->d_rowmap, s->total_rows, s->max_ld,
                                            s->stream);
    if (e != hipSuccess) return server_fail(s, e, "aco_server_step");
    ++s->ticks;
    for (int idx : s->running) {
        Slot& sl = s->slots[idx];
        if (++sl.iters_queued == sl.iters_total) s->dirty = true;  // leaves after this tick
    }
    return ACO_OK;
}

aco_status aco_server_collect(aco_server* s, int32_t* slots_out, int64_t* ids_out, int32_t max,
                              int32_t* count_out) {
    if (aco_status st = server_usable(s)) return st;
    if (!count_out || (max > 0 && (!slots_out || !ids_out)))
        return fail(ACO_ERR_INVALID, "NULL output");
    *count_out = 0;
    const hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return server_fail(s, e, "aco_server_collect");
    for (size_t i = 0; i < s->slots.size() && *count_out < max; ++i) {
        Slot& sl = s->slots[i];
        if (sl.state == kRunning && sl.iters_queued == sl.iters_total) {
            sl.state = kDone;
            slots_out[*count_out] = (int32_t)i;
            ids_out[*count_out] = sl.request_id;
            ++*count_out;
        }
    }
    return ACO_OK;
}

aco_status aco_server_result(aco_server* s, int32_t slot, uint16_t* best_tour_host,
                             int64_t* best_len_host) {
    if (aco_status st = server_usable(s)) return st;
    if (slot < 0 || slot >= (int32_t)s->slots.size() || s->slots[slot].state != kDone)
        return fail(ACO_ERR_STATE, "slot holds no finished request");
    const aco::Colony& c = s->slots[slot].col;
    hipError_t e = hipSuccess;
    if (best_len_host) e = hipMemcpy(best_len_host, c.best_len, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && best_tour_host)
        e = hipMemcpy(best_tour_host, c.best_tour, ((size_t)c.n + 1) * sizeof(uint16_t),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) return server_fail(s, e, "aco_server_result");
    return ACO_OK;
}

aco_status aco_server_read_tau(aco_server* s, int32_t slot, float* tau_host) {
    if (aco_status st = server_usable(s)) return st;
    if (slot < 0 || slot >= (int32_t)s->slots.size() || s->slots[slot].state != kDone)
        return fail(ACO_ERR_STATE, "slot holds no finished request");
    if (!tau_host) return fail(ACO_ERR_INVALID, "tau_host is NULL");
    const aco::Colony& c = s->slots[slot].col;
    const hipError_t e =
        hipMemcpy2D(tau_host, (size_t)c.n * sizeof(float), c.tau, (size_t)c.ld * sizeof(float),
                    (size_t)c.n * sizeof(float), (size_t)c.n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return server_fail(s, e, "aco_server_read_tau");
    return ACO_OK;
}

aco_status aco_server_release(aco_server* s, int32_t slot) {
    if (aco_status st = server_usable(s)) return st;
    if (slot < 0 || slot >= (int32_t)s->slots.size() || s->slots[slot].state != kDone)
        return fail(ACO_ERR_STATE, "slot holds no finished request");
    Slot& sl = s->slots[slot];
    pool_free(s, sl.off, sl.bytes);
    sl.state = kFree;
    sl.request_id = -1;
    return ACO_OK;
}

aco_status aco_server_stats(aco_server* s, int32_t* running, int32_t* initialising,
                            int32_t* finished, size_t* free_bytes, size_t* largest_free_block,
                            uint64_t* ticks) {
    if (aco_status st = server_usable(s)) return st;
    int r = 0, in = 0, f = 0;
    size_t fb = 0;
    for (const Slot& sl : s->slots) {
        r += sl.state == kRunning;
        in += sl.state == kInit;
        f += sl.state == kDone;
    }
    for (const auto& kv : s->free_blocks) fb += kv.second;
    if (running) *running = r;
    if (initialising) *initialising = in;
    if (finished) *finished = f;
    if (free_bytes) *free_bytes = fb;
    if (largest_free_block) *largest_free_block = largest_free(s);
    if (ticks) *ticks = s->ticks;
    return ACO_OK;
}

void aco_server_destroy(aco_server* s) {
    if (!s) return;
    if (s->init_stream) (void)hipStreamSynchronize(s->init_stream);
    if (s->stream || s->init_stream) (void)hipStreamSynchronize(s->stream);
    for (Slot& sl : s->slots)
        if (sl.ready) (void)hipEventDestroy(sl.ready);
    if (s->init_stream) (void)hipStreamDestroy(s->init_stream);
    delete s;
}

}  // extern "C"
