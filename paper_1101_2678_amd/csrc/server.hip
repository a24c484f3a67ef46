// server.hip -- continuous batching of independent Ant System solves.
//
// A server owns a caller-provided device pool.  A request (an instance and a
// number of iterations) is admitted when a slot is free and the pool has a
// free block for the request's whole workspace (first fit; the footprint is
// aco_workspace_bytes without the atomic part).  Its distances are uploaded
// and its colony initialised on the server's admission stream; it joins the
// running set of its size class at the first tick after that work has
// finished.
//
// Each size class has its own running set, device tables, stream and tick:
// a tick advances every running request of the class by one AS iteration with
// the batched kernels (one construction launch over all their ants, one
// best-so-far launch, one gather launch over all their rows).  Classes tick
// independently and concurrently, so a 100-city request is not paced by the
// iterations of a 3000-city one, and requests that arrive while others run
// share the device.  aco_server_step never blocks: it completes the ticks
// that have finished, lets ready requests join, and starts the next tick of
// every idle class.  A request whose iterations are done leaves its set; its
// result stays readable until the slot is released.  Every request computes
// exactly what a context of its own computes.
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
    uint32_t iters_total = 0, iters_done = 0;
    int64_t request_id = -1;
    int cls = 0;
    bool reported = false;
    hipEvent_t ready = nullptr;  // initialisation finished
};

// One size class: its running set, device tables and tick stream.
struct SizeClass {
    int max_n = 0;
    aco::Colony* d_cols = nullptr;
    uint32_t* d_antmap = nullptr;
    uint32_t* d_rowmap = nullptr;
    std::vector<int> running;  // slot indices in launch order (largest n first)
    std::vector<aco::Colony> h_cols;
    std::vector<uint32_t> h_antmap, h_rowmap;  // host copies kept alive for async uploads
    int total_ants = 0, total_rows = 0, run_max_n = 0, run_max_ld = 0;
    bool dirty = false, in_flight = false;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint64_t ticks = 0;
};

}  // namespace

struct aco_server {
    char* pool = nullptr;
    size_t pool_bytes = 0;
    std::map<size_t, size_t> free_blocks;  // offset -> size, coalesced
    std::vector<Slot> slots;
    std::vector<SizeClass> classes;
    int max_ants = 0, max_rows = 0;
    int cus = 0;            // compute units of the device
    size_t lds_per_cu = 0;  // LDS bytes per compute unit
    hipStream_t init_stream = nullptr;
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

size_t class_table_bytes(int32_t max_slots, int32_t max_ants, int32_t max_rows) {
    const size_t a = aco::host::kAlign;
    return aco::host::round_up((size_t)max_slots * sizeof(aco::Colony), a) +
           aco::host::round_up((size_t)max_ants * sizeof(uint32_t), a) +
           aco::host::round_up((size_t)max_rows * sizeof(uint32_t), a);
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

int class_of(const aco_server* s, int n) {
    for (size_t c = 0; c < s->classes.size(); ++c)
        if (n <= s->classes[c].max_n) return (int)c;
    return (int)s->classes.size() - 1;
}

// Rebuilds the tables of class c from its running slots.  Only called when
// no tick of the class is in flight; the uploads are ordered before the next
// tick on the class stream.
hipError_t rebuild_class(aco_server* s, int c) {
    SizeClass& k = s->classes[c];
    std::vector<int> run;
    for (size_t i = 0; i < s->slots.size(); ++i) {
        const Slot& sl = s->slots[i];
        if (sl.cls == c && sl.state == kRunning && sl.iters_done < sl.iters_total)
            run.push_back((int)i);
    }
    std::stable_sort(run.begin(), run.end(),
                     [&](int a, int b) { return s->slots[a].col.n > s->slots[b].col.n; });
    k.h_cols.clear();
    k.h_antmap.clear();
    k.h_rowmap.clear();
    int max_n = 0, max_ld = 0;
    for (size_t pos = 0; pos < run.size(); ++pos) {
        const aco::Colony& col = s->slots[run[pos]].col;
        k.h_cols.push_back(col);
        for (int a = 0; a < col.m; ++a) k.h_antmap.push_back(((uint32_t)pos << 16) | (uint32_t)a);
        for (int r = 0; r < col.n; ++r) k.h_rowmap.push_back(((uint32_t)pos << 16) | (uint32_t)r);
        max_n = std::max(max_n, col.n);
        max_ld = std::max(max_ld, col.ld);
    }
    hipError_t e = hipSuccess;
    if (!k.h_cols.empty())
        e = hipMemcpyAsync(k.d_cols, k.h_cols.data(), sizeof(aco::Colony) * k.h_cols.size(),
                           hipMemcpyHostToDevice, k.stream);
    if (e == hipSuccess && !k.h_antmap.empty())
        e = hipMemcpyAsync(k.d_antmap, k.h_antmap.data(), sizeof(uint32_t) * k.h_antmap.size(),
                           hipMemcpyHostToDevice, k.stream);
    if (e == hipSuccess && !k.h_rowmap.empty())
        e = hipMemcpyAsync(k.d_rowmap, k.h_rowmap.data(), sizeof(uint32_t) * k.h_rowmap.size(),
                           hipMemcpyHostToDevice, k.stream);
    if (e != hipSuccess) return e;
    k.running = run;
    k.total_ants = (int)k.h_antmap.size();
    k.total_rows = (int)k.h_rowmap.size();
    k.run_max_n = max_n;
    k.run_max_ld = max_ld;
    k.dirty = false;
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t aco_server_table_bytes(int32_t max_slots, int32_t max_ants, int32_t max_rows,
                              int32_t num_classes) {
    if (max_slots < 1 || max_slots > 65535 || max_ants < 1 || max_rows < 1 || num_classes < 1 ||
        num_classes > 8)
        return 0;
    return (size_t)num_classes * class_table_bytes(max_slots, max_ants, max_rows);
}

aco_status aco_server_create(aco_server** out, void* d_pool, size_t pool_bytes, int32_t max_slots,
                             int32_t max_ants, int32_t max_rows, int32_t num_classes,
                             const int32_t* class_max_n) {
    aco::host::g_error.clear();
    if (!out) return fail(ACO_ERR_INVALID, "out is NULL");
    *out = nullptr;
    const size_t head = aco_server_table_bytes(max_slots, max_ants, max_rows, num_classes);
    if (head == 0)
        return fail(ACO_ERR_INVALID,
                    "max_slots in [1, 65535], max_ants and max_rows >= 1, 1 <= num_classes <= 8");
    if (!class_max_n) return fail(ACO_ERR_INVALID, "class_max_n is NULL");
    for (int c = 0; c < num_classes; ++c)
        if (class_max_n[c] < 3 || (c > 0 && class_max_n[c] <= class_max_n[c - 1]))
            return fail(ACO_ERR_INVALID, "class_max_n must be increasing and >= 3");
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
    s->classes.resize(num_classes);
    const size_t a = aco::host::kAlign;
    const size_t per = class_table_bytes(max_slots, max_ants, max_rows);
    hipError_t e = aco::host::device_shape(&s->cus, &s->lds_per_cu);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->init_stream, hipStreamNonBlocking);
    for (int c = 0; c < num_classes; ++c) {
        SizeClass& k = s->classes[c];
        char* base = s->pool + (size_t)c * per;
        k.max_n = class_max_n[c];
        k.d_cols = reinterpret_cast<aco::Colony*>(base);
        k.d_antmap = reinterpret_cast<uint32_t*>(
            base + aco::host::round_up((size_t)max_slots * sizeof(aco::Colony), a));
        k.d_rowmap = reinterpret_cast<uint32_t*>(
            reinterpret_cast<char*>(k.d_antmap) +
            aco::host::round_up((size_t)max_ants * sizeof(uint32_t), a));
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&k.done, hipEventDisableTiming);
    }
    if (pool_bytes > head) s->free_blocks[head] = pool_bytes - head;
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
    int dep_emin = 0;
    if (!aco::host::dist_valid(dist_host, p->n, p->m, &why, &dep_emin))
        return fail(ACO_ERR_INVALID, why);
    const int cls = class_of(s, p->n);
    int free_slot = -1;
    int class_ants = 0, class_rows = 0;
    for (size_t i = 0; i < s->slots.size(); ++i) {
        const Slot& sl = s->slots[i];
        if (sl.state == kFree && free_slot < 0) free_slot = (int)i;
        if ((sl.state == kInit || sl.state == kRunning) && sl.cls == cls) {
            class_ants += sl.col.m;
            class_rows += sl.col.n;
        }
    }
    if (free_slot < 0) return fail(ACO_ERR_STATE, "no free slot");
    if (class_ants + p->m > s->max_ants || class_rows + p->n > s->max_rows)
        return fail(ACO_ERR_STATE, "the size class would exceed max_ants or max_rows");
    const aco::host::Layout L = aco::host::make_layout(*p);
    size_t off = 0;
    if (!pool_alloc(s, L.base_end, &off)) return fail(ACO_ERR_NOMEM, "no free pool block large enough");
    Slot& sl = s->slots[free_slot];
    sl.col = aco::host::carve(s->pool + off, L, *p, false, dep_emin, aco::host::tile_for(p->n));
    sl.off = off;
    sl.bytes = L.base_end;
    sl.iters_total = iters;
    sl.iters_done = 0;
    sl.request_id = request_id;
    sl.cls = cls;
    sl.reported = false;
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
    hipError_t e = hipSuccess;
    // Requests whose initialisation has finished join their class.
    for (Slot& sl : s->slots) {
        if (sl.state != kInit) continue;
        const hipError_t q = hipEventQuery(sl.ready);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return server_fail(s, q, "aco_server_step");
        sl.state = kRunning;
        s->classes[sl.cls].dirty = true;
    }
    int running = 0;
    for (size_t c = 0; c < s->classes.size(); ++c) {
        SizeClass& k = s->classes[c];
        if (k.in_flight) {
            const hipError_t q = hipEventQuery(k.done);
            if (q == hipErrorNotReady) {
                running += (int)k.running.size();
                continue;
            }
            if (q != hipSuccess) return server_fail(s, q, "aco_server_step");
            k.in_flight = false;
            for (int idx : k.running) {
                Slot& sl = s->slots[idx];
                if (++sl.iters_done == sl.iters_total) {
                    sl.state = kDone;
                    k.dirty = true;
                }
            }
        }
        if (k.dirty) e = rebuild_class(s, (int)c);
        if (e != hipSuccess) return server_fail(s, e, "aco_server_step");
        if (k.running.empty()) continue;
        e = aco::launch_construct_batch(
            k.d_cols, k.d_antmap, k.total_ants, k.run_max_n,
            aco::batch_lds_bytes(k.run_max_n, aco::batch_default_cap(k.total_ants, s->cus),
                                 s->lds_per_cu),
            k.stream);
        if (e == hipSuccess) e = aco::launch_best_batch(k.d_cols, (int)k.running.size(), k.stream);
        if (e == hipSuccess)
            e = aco::launch_update_gather_batch(k.d_cols, k.d_rowmap, k.total_rows, k.run_max_ld,
                                                k.stream);
        if (e == hipSuccess) e = hipEventRecord(k.done, k.stream);
        if (e != hipSuccess) return server_fail(s, e, "aco_server_step");
        k.in_flight = true;
        ++k.ticks;
        running += (int)k.running.size();
    }
    if (running_out) *running_out = running;
    return ACO_OK;
}

aco_status aco_server_collect(aco_server* s, int32_t* slots_out, int64_t* ids_out, int32_t max,
                              int32_t* count_out) {
    if (aco_status st = server_usable(s)) return st;
    if (!count_out || (max > 0 && (!slots_out || !ids_out)))
        return fail(ACO_ERR_INVALID, "NULL output");
    *count_out = 0;
    for (size_t i = 0; i < s->slots.size() && *count_out < max; ++i) {
        Slot& sl = s->slots[i];
        if (sl.state == kDone && !sl.reported) {
            sl.reported = true;
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
    size_t fb = 0, lb = 0;
    uint64_t t = 0;
    for (const Slot& sl : s->slots) {
        r += sl.state == kRunning;
        in += sl.state == kInit;
        f += sl.state == kDone;
    }
    for (const auto& kv : s->free_blocks) {
        fb += kv.second;
        lb = std::max(lb, kv.second);
    }
    for (const SizeClass& k : s->classes) t += k.ticks;
    if (running) *running = r;
    if (initialising) *initialising = in;
    if (finished) *finished = f;
    if (free_bytes) *free_bytes = fb;
    if (largest_free_block) *largest_free_block = lb;
    if (ticks) *ticks = t;
    return ACO_OK;
}

void aco_server_destroy(aco_server* s) {
    if (!s) return;
    if (s->init_stream) (void)hipStreamSynchronize(s->init_stream);
    for (SizeClass& k : s->classes) {
        if (k.stream) (void)hipStreamSynchronize(k.stream);
        if (k.done) (void)hipEventDestroy(k.done);
        if (k.stream) (void)hipStreamDestroy(k.stream);
    }
    for (Slot& sl : s->slots)
        if (sl.ready) (void)hipEventDestroy(sl.ready);
    if (s->init_stream) (void)hipStreamDestroy(s->init_stream);
    delete s;
}

}  // extern "C"
