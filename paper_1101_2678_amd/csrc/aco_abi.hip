// aco_abi.hip -- the C ABI of libaco (declared in include/aco.h): argument
// validation, workspace carving, the per-context state machine and error
// reporting.  All arithmetic of the method runs in the kernels of
// construct.hip and update.hip; this file only moves bytes and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "aco.h"
#include "aco_ctx.hpp"
#include "aco_host.hpp"
#include "aco_state.hpp"
#include "nn.hpp"
#include "product.hpp"


namespace aco {
namespace host {

thread_local std::string g_error;

aco_status fail(aco_status s, const std::string& why) {
    g_error = why;
    return s;
}

aco_status device_fail(bool* poisoned, hipError_t e, const char* where) {
    if (poisoned) *poisoned = true;
    return fail(ACO_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// A stream handle must belong to the HIP runtime this library runs on and to
// `device`.  Work enqueued on a handle the runtime does not know would not be
// ordered with the library's other calls on that stream, so such a handle is
// refused up front.  NULL (the default stream) is always accepted.
aco_status stream_on_device(void* hip_stream, int device, const char* where) {
    if (!hip_stream) return ACO_OK;
    hipDevice_t owner = -1;
    const hipError_t e = hipStreamGetDevice(static_cast<hipStream_t>(hip_stream), &owner);
    if (e != hipSuccess) {
        // The runtime also keeps the failure as this thread's last error; the
        // launch checks (hipGetLastError after each launch) of the next call
        // would report it as their own, so it is consumed here.
        (void)hipGetLastError();
        return fail(ACO_ERR_DEVICE, std::string(where) +
                                        ": the stream is not a stream of this HIP runtime (" +
                                        hipGetErrorString(e) + ")");
    }
    if ((int)owner != device)
        return fail(ACO_ERR_INVALID, std::string(where) + ": the stream belongs to device " +
                                         std::to_string((int)owner) + ", not the current device " +
                                         std::to_string(device));
    return ACO_OK;
}

bool params_valid(const aco_params* p, std::string* why) {
    if (!p) return (*why = "params is NULL", false);
    if (p->n < 3 || p->n > kMaxCities) return (*why = "n must be in [3, 4096]", false);
    if (p->m < 1 || p->m > 65535) return (*why = "m must be in [1, 65535]", false);
    if (p->alpha < 0 || p->alpha > 2) return (*why = "alpha must be 0, 1 or 2", false);
    if (p->beta < 0 || p->beta > 4) return (*why = "beta must be in [0, 4]", false);
    if (!(p->rho > 0.0f && p->rho <= 1.0f)) return (*why = "rho must be in (0, 1]", false);
    return true;
}

Layout make_layout(const aco_params& p) {
    Layout L{};
    L.ld = (int32_t)round_up((size_t)p.n, 64);
    L.tp = (int32_t)round_up((size_t)p.n + 1, 64);
    L.mp = (int32_t)round_up((size_t)p.m, 64);
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t o = off;
        off = round_up(off + bytes, kAlign);
        return o;
    };
    const size_t cells = (size_t)p.n * L.ld;
    L.tau = take(cells * sizeof(float));
    L.choice = take(cells * sizeof(float));
    L.dist = take(cells * sizeof(int32_t));
    L.tours = take((size_t)p.m * L.tp * sizeof(uint16_t));
    L.succ = take((size_t)p.n * L.mp * sizeof(uint16_t));
    L.pred = take((size_t)p.n * L.mp * sizeof(uint16_t));
    L.lens = take((size_t)p.m * sizeof(int64_t));
    L.dep = take((size_t)p.m * sizeof(float));
    L.best_len = take(sizeof(int64_t));
    L.best_tour = take((size_t)L.tp * sizeof(uint16_t));
    L.cnn = take(sizeof(int64_t));
    L.tau0 = take(sizeof(float));
    L.iter = take(sizeof(uint32_t));
    L.base_end = off;
    L.delta = take(cells * sizeof(double));
    L.atomic_end = off;
    return L;
}

// Distances must describe a symmetric complete graph (Section II) with
// positive off-diagonal weights.  The deposit sums of the update are exact
// in binary64 only if the deposits 1/C^k span few binades: with
// LB <= C^k <= UB (each city contributes half of its two cheapest / two
// dearest incident edges) we need bits(m) + bits(UB/LB) + 1 + 24 <= 53.
bool dist_valid(const int32_t* d, int n, int m, std::string* why, int* dep_emin) {
    double lb = 0.0, ub = 0.0;
    for (int i = 0; i < n; ++i) {
        if (d[(size_t)i * n + i] != 0) return (*why = "distance matrix diagonal must be 0", false);
        int64_t lo1 = INT64_MAX, lo2 = INT64_MAX, hi1 = -1, hi2 = -1;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const int32_t v = d[(size_t)i * n + j];
            if (v < 1) return (*why = "off-diagonal distances must be >= 1", false);
            if (v != d[(size_t)j * n + i]) return (*why = "distance matrix must be symmetric", false);
            if (v < lo1) { lo2 = lo1; lo1 = v; } else if (v < lo2) lo2 = v;
            if (v > hi1) { hi2 = hi1; hi1 = v; } else if (v > hi2) hi2 = v;
        }
        lb += 0.5 * (double)(lo1 + lo2);
        ub += 0.5 * (double)(hi1 + hi2);
    }
    int mbits = 0;
    while ((1LL << mbits) < (long long)m) ++mbits;
    const int spread = (int)std::ceil(std::log2(ub / lb)) + 1;
    if (mbits + spread + 24 > 53)
        return (*why = "tour lengths span too many binades for exact binary64 deposit sums", false);
    if (dep_emin) {
        // every C^k <= UB, so every deposit fl32(1/C^k) >= fl32(1/UB): its
        // exponent field bounds theirs from below (the fixed-point scale of
        // the update's accumulators)
        const float dmin = (float)(1.0 / ub);
        uint32_t bits;
        std::memcpy(&bits, &dmin, sizeof bits);
        *dep_emin = (int)((bits >> 23) & 0xFFu);
    }
    return true;
}

Colony carve(char* base, const Layout& L, const aco_params& p, bool with_delta, int dep_emin,
             int tile, int waves) {
    Colony col{};
    col.n = p.n;
    col.m = p.m;
    col.ld = L.ld;
    col.tp = L.tp;
    col.mp = L.mp;
    col.alpha = p.alpha;
    col.beta = p.beta;
    col.rho = p.rho;
    col.seed = p.seed;
    col.tau = reinterpret_cast<float*>(base + L.tau);
    col.choice = reinterpret_cast<float*>(base + L.choice);
    col.dist = reinterpret_cast<int32_t*>(base + L.dist);
    col.tours = reinterpret_cast<uint16_t*>(base + L.tours);
    col.succ = reinterpret_cast<uint16_t*>(base + L.succ);
    col.pred = reinterpret_cast<uint16_t*>(base + L.pred);
    col.lens = reinterpret_cast<int64_t*>(base + L.lens);
    col.dep = reinterpret_cast<float*>(base + L.dep);
    col.best_len = reinterpret_cast<int64_t*>(base + L.best_len);
    col.best_tour = reinterpret_cast<uint16_t*>(base + L.best_tour);
    col.cnn = reinterpret_cast<int64_t*>(base + L.cnn);
    col.tau0 = reinterpret_cast<float*>(base + L.tau0);
    col.iter_dev = reinterpret_cast<uint32_t*>(base + L.iter);
    col.delta = with_delta ? reinterpret_cast<double*>(base + L.delta) : nullptr;
    col.tile = tile;
    col.waves = waves;
    col.dep_emin = dep_emin;
    return col;
}

hipError_t upload_and_init(const Colony& col, const int32_t* dist_host, size_t base_bytes,
                           hipStream_t stream) {
    hipError_t e = hipMemsetAsync(col.tau, 0, base_bytes, stream);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(col.dist, (size_t)col.ld * sizeof(int32_t), dist_host,
                             (size_t)col.n * sizeof(int32_t), (size_t)col.n * sizeof(int32_t),
                             (size_t)col.n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_init(col, stream);
    return e;
}

// Construction shape per instance size: the tile (cities per lane) and the
// wavefronts per ant.  Default: 4 cities per lane up to n = 256, 8 above,
// one wavefront per ant (single-instance construction with m = n on MI355X:
// tile 4 5-7% faster at n = 64..256, tile 8 7-12% faster at 320..1024, two
// or four wavefronts per ant 5-30% slower).  The table is filled once, on
// first use, by a function-local static (thread-safe initialisation);
// changing it while other threads read it is not supported.
namespace {
constexpr int kTile4Max = 256;

struct Shape {
    int8_t tile, waves;
};

void fill_default_tiles(Shape* t) {
    for (int n = 0; n <= kMaxCities; ++n) t[n] = Shape{(int8_t)(n <= kTile4Max ? 4 : 8), 1};
}

Shape* tile_table() {
    static Shape* const table = [] {
        static Shape t[kMaxCities + 1];
        fill_default_tiles(t);
        return t;
    }();
    return table;
}
}  // namespace

void reset_tiles() { fill_default_tiles(tile_table()); }

hipError_t device_shape(int* cus, size_t* lds_per_cu) {
    int dev = 0, n_cu = 0, lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    if (e != hipSuccess) return e;
    *cus = n_cu;
    *lds_per_cu = (size_t)lds;
    return hipSuccess;
}

int tile_for(int n) {
    return (n >= 0 && n <= kMaxCities) ? tile_table()[n].tile : 8;
}

int waves_for(int n) {
    return (n >= 0 && n <= kMaxCities) ? tile_table()[n].waves : 1;
}

bool shape_supported(int tile, int waves, int n) {
    return waves == 1 ? tile_supported(tile, n) : split_supported(tile, waves, n);
}

bool set_shape_range(int lo, int hi, int tile, int waves) {
    if (lo < 1 || hi > kMaxCities || lo > hi) return false;
    for (int n = lo; n <= hi; ++n)
        if (!shape_supported(tile, waves, n)) return false;
    Shape* t = tile_table();
    for (int n = lo; n <= hi; ++n) t[n] = Shape{(int8_t)tile, (int8_t)waves};
    return true;
}

bool set_tile_range(int lo, int hi, int tile) { return set_shape_range(lo, hi, tile, 1); }

}  // namespace host
}  // namespace aco

namespace {

using aco::host::fail;
using aco::host::g_error;

aco_status device_fail(aco_ctx* c, hipError_t e, const char* where) {
    return aco::host::device_fail(c ? &c->poisoned : nullptr, e, where);
}

aco_status usable(aco_ctx* c) {
    if (!c) return fail(ACO_ERR_INVALID, "context is NULL");
    if (c->poisoned) return fail(ACO_ERR_STATE, "context poisoned by an earlier device error");
    return ACO_OK;
}

aco_status sync_ctx(aco_ctx* c, const char* where) {
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(c, e, where);
    return ACO_OK;
}

}  // namespace

namespace aco {
namespace host {

aco_status update_ready(aco_ctx* c) {
    if (aco_status s = usable(c)) return s;
    if (!c->pending) return fail(ACO_ERR_STATE, "aco_update needs a preceding aco_construct");
    return ACO_OK;
}

aco_status enqueue_update(aco_ctx* c, aco_update_kind kind, double* delta) {
    // the update kernels also keep the best-so-far tour
    hipError_t e;
    if (kind == ACO_UPDATE_GATHER) {
        e = launch_update_gather(c->col, c->stream);
    } else {
        Colony col = c->col;
        if (delta) col.delta = delta;
        e = launch_update_atomic(col, kind == ACO_UPDATE_ATOMIC, c->stream);
    }
    if (e != hipSuccess) return ::device_fail(c, e, "aco_update");
    c->pending = false;
    c->next_iter = c->pending_iter + 1;
    return ACO_OK;
}

}  // namespace host
}  // namespace aco

extern "C" {

const char* aco_status_str(aco_status s) {
    switch (s) {
        case ACO_OK: return "ok";
        case ACO_ERR_INVALID: return "invalid argument";
        case ACO_ERR_NOMEM: return "workspace too small or misaligned";
        case ACO_ERR_DEVICE: return "device error";
        case ACO_ERR_STATE: return "invalid call order or poisoned context";
    }
    return "unknown status";
}

const char* aco_last_error(void) { return g_error.c_str(); }

size_t aco_workspace_bytes(const aco_params* p, int32_t with_atomic) {
    std::string why;
    if (!aco::host::params_valid(p, &why)) return 0;
    const aco::host::Layout L = aco::host::make_layout(*p);
    return with_atomic ? L.atomic_end : L.base_end;
}

aco_status aco_init(aco_ctx** out, const aco_params* p, const int32_t* dist_host,
                    void* d_workspace, size_t ws_bytes, void* hip_stream) {
    g_error.clear();
    if (!out) return fail(ACO_ERR_INVALID, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!aco::host::params_valid(p, &why)) return fail(ACO_ERR_INVALID, why);
    if (!dist_host) return fail(ACO_ERR_INVALID, "dist_host is NULL");
    int dep_emin = 0;
    if (!aco::host::dist_valid(dist_host, p->n, p->m, &why, &dep_emin))
        return fail(ACO_ERR_INVALID, why);
    const aco::host::Layout L = aco::host::make_layout(*p);
    if (!d_workspace || ((uintptr_t)d_workspace % aco::host::kAlign) != 0)
        return fail(ACO_ERR_NOMEM, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < L.base_end)
        return fail(ACO_ERR_NOMEM, "workspace smaller than aco_workspace_bytes(p, 0)");

    int device = 0;
    if (hipGetDevice(&device) != hipSuccess)
        return fail(ACO_ERR_DEVICE, "aco_init: no current HIP device");
    if (aco_status s = aco::host::stream_on_device(hip_stream, device, "aco_init")) return s;

    aco_ctx* c = new (std::nothrow) aco_ctx();
    if (!c) return fail(ACO_ERR_NOMEM, "host allocation failed");
    c->device = device;
    c->scratch_err = aco::host::noalloc_scratch(device, &c->scratch);
    c->has_atomic = ws_bytes >= L.atomic_end;
    c->col = aco::host::carve(static_cast<char*>(d_workspace), L, *p, c->has_atomic, dep_emin,
                              aco::host::tile_for(p->n), aco::host::waves_for(p->n));
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws_bytes = ws_bytes;
    hipError_t e = aco::host::upload_and_init(c->col, dist_host, L.base_end, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        aco_status s = device_fail(c, e, "aco_init");
        delete c;
        return s;
    }
    *out = c;
    return ACO_OK;
}

aco_status aco_set_tile(int32_t n_lo, int32_t n_hi, int32_t cities_per_lane) {
    if (!aco::host::set_tile_range(n_lo, n_hi, cities_per_lane))
        return fail(ACO_ERR_INVALID,
                    "tile must be 8 (any n) or 4 (n <= 1024) over 1 <= n_lo <= n_hi <= 4096");
    return ACO_OK;
}

aco_status aco_set_shape(int32_t n_lo, int32_t n_hi, int32_t cities_per_lane,
                         int32_t waves_per_ant) {
    if (!aco::host::set_shape_range(n_lo, n_hi, cities_per_lane, waves_per_ant))
        return fail(ACO_ERR_INVALID,
                    "shape not supported over the range: 1 wavefront per ant with tile 8 (any "
                    "n) or 4 (n <= 1024); 2 or 4 wavefronts only for n <= 1024 with at least "
                    "as many passes of 64 * tile cities (tile 8: 2 waves; tile 4: 2 waves, or "
                    "4 waves at 4 passes)");
    return ACO_OK;
}

int32_t aco_get_tile(int32_t n) { return aco::host::tile_for(n); }

int32_t aco_get_waves(int32_t n) { return aco::host::waves_for(n); }

void aco_reset_tiles(void) { aco::host::reset_tiles(); }

aco_status aco_construct(aco_ctx* c, uint32_t iter) {
    if (aco_status s = usable(c)) return s;
    const hipError_t e = aco::launch_construct(c->col, iter, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "aco_construct");
    c->pending = true;
    c->pending_iter = iter;
    return ACO_OK;
}

aco_status aco_update(aco_ctx* c, aco_update_kind kind) {
    if (aco_status s = aco::host::update_ready(c)) return s;
    if (kind != ACO_UPDATE_GATHER && kind != ACO_UPDATE_ATOMIC && kind != ACO_UPDATE_ATOMIC_DIRECT)
        return fail(ACO_ERR_INVALID, "unknown update kind");
    if (kind != ACO_UPDATE_GATHER && !c->has_atomic)
        return fail(ACO_ERR_INVALID, "workspace has no room for the atomic update");
    return aco::host::enqueue_update(c, kind, nullptr);
}

static aco_status solve_with(aco_ctx* c, uint32_t iters, aco_update_kind kind,
                             aco_status (*construct)(aco_ctx*, uint32_t),
                             uint16_t* best_tour_host, int64_t* best_len_host) {
    if (aco_status s = usable(c)) return s;
    if (kind != ACO_UPDATE_GATHER && kind != ACO_UPDATE_ATOMIC && kind != ACO_UPDATE_ATOMIC_DIRECT)
        return fail(ACO_ERR_INVALID, "unknown update kind");
    if (kind != ACO_UPDATE_GATHER && !c->has_atomic)
        return fail(ACO_ERR_INVALID, "workspace has no room for the atomic update");
    for (uint32_t i = 0; i < iters; ++i) {
        if (aco_status s = construct(c, c->next_iter)) return s;
        if (aco_status s = aco_update(c, kind)) return s;
    }
    return aco_read_best(c, best_tour_host, best_len_host);
}

aco_status aco_solve(aco_ctx* c, uint32_t iters, aco_update_kind kind, uint16_t* best_tour_host,
                     int64_t* best_len_host) {
    return solve_with(c, iters, kind, aco_construct, best_tour_host, best_len_host);
}

aco_status aco_construct_product(aco_ctx* c, uint32_t iter) {
    if (aco_status s = usable(c)) return s;
    const hipError_t e = aco::launch_construct_product(c->col, iter, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "aco_construct_product");
    c->pending = true;
    c->pending_iter = iter;
    return ACO_OK;
}

aco_status aco_solve_product(aco_ctx* c, uint32_t iters, aco_update_kind kind,
                             uint16_t* best_tour_host, int64_t* best_len_host) {
    return solve_with(c, iters, kind, aco_construct_product, best_tour_host, best_len_host);
}

aco_status aco_test_product_select(int32_t n, int32_t count, const float* rows_dev,
                                   const uint8_t* feasible_dev, const float* u_dev,
                                   int32_t* out_dev, void* hip_stream) {
    if (n < 1 || n > aco::kMaxCities) return fail(ACO_ERR_INVALID, "n must be in [1, 4096]");
    if (count < 0) return fail(ACO_ERR_INVALID, "count must be >= 0");
    if (count > 0 && (!rows_dev || !feasible_dev || !u_dev || !out_dev))
        return fail(ACO_ERR_INVALID, "NULL device pointer");
    if (((uintptr_t)rows_dev % 16) != 0)
        return fail(ACO_ERR_INVALID, "rows must be 16-byte aligned");
    const hipError_t e = aco::launch_test_product_select(
        n, count, rows_dev, feasible_dev, u_dev, out_dev, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return device_fail(nullptr, e, "aco_test_product_select");
    return ACO_OK;
}

size_t aco_nn_workspace_bytes(int32_t n, int32_t nn) {
    if (n < 3 || n > aco::kMaxCities || nn < 1 || nn > aco::kMaxNn || nn > n - 1) return 0;
    return aco::nn_table_bytes(n, nn);
}

aco_status aco_nn_attach(aco_ctx* c, int32_t nn, void* d_nn_workspace, size_t bytes) {
    if (aco_status s = usable(c)) return s;
    if (nn < 1 || nn > aco::kMaxNn || nn > c->col.n - 1)
        return fail(ACO_ERR_INVALID, "nn must be in [1, min(64, n - 1)]");
    if (!d_nn_workspace || ((uintptr_t)d_nn_workspace % aco::host::kAlign) != 0)
        return fail(ACO_ERR_NOMEM, "nn workspace must be a 256-byte aligned device pointer");
    if (bytes < aco::nn_table_bytes(c->col.n, nn))
        return fail(ACO_ERR_NOMEM, "nn workspace smaller than aco_nn_workspace_bytes(n, nn)");
    const aco::NnTables t = aco::nn_carve(static_cast<char*>(d_nn_workspace), c->col.n, nn);
    const hipError_t e = aco::launch_nn_lists(c->col, t, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "aco_nn_attach");
    c->nn = t;
    return ACO_OK;
}

aco_status aco_construct_nn(aco_ctx* c, uint32_t iter) {
    if (aco_status s = usable(c)) return s;
    if (c->nn.nn == 0) return fail(ACO_ERR_STATE, "aco_construct_nn needs aco_nn_attach first");
    const hipError_t e = aco::launch_construct_nn(c->col, c->nn, iter, c->stream);
    if (e != hipSuccess) return device_fail(c, e, "aco_construct_nn");
    c->pending = true;
    c->pending_iter = iter;
    return ACO_OK;
}

aco_status aco_solve_nn(aco_ctx* c, uint32_t iters, aco_update_kind kind,
                        uint16_t* best_tour_host, int64_t* best_len_host) {
    if (aco_status s = usable(c)) return s;
    if (c->nn.nn == 0) return fail(ACO_ERR_STATE, "aco_solve_nn needs aco_nn_attach first");
    return solve_with(c, iters, kind, aco_construct_nn, best_tour_host, best_len_host);
}

aco_status aco_read_nn_lists(aco_ctx* c, uint16_t* lists_host) {
    if (aco_status s = usable(c)) return s;
    if (c->nn.nn == 0) return fail(ACO_ERR_STATE, "no candidate lists attached");
    if (!lists_host) return fail(ACO_ERR_INVALID, "host pointer is NULL");
    if (aco_status s = sync_ctx(c, "aco_read_nn_lists")) return s;
    // one contiguous copy of the padded table, repacked on the host
    std::vector<uint16_t> padded((size_t)c->col.n * c->nn.kp);
    const hipError_t e = hipMemcpy(padded.data(), c->nn.nnl, padded.size() * sizeof(uint16_t),
                                   hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(c, e, "aco_read_nn_lists");
    for (int i = 0; i < c->col.n; ++i)
        std::memcpy(lists_host + (size_t)i * c->nn.nn, padded.data() + (size_t)i * c->nn.kp,
                    (size_t)c->nn.nn * sizeof(uint16_t));
    return ACO_OK;
}

aco_status aco_read_best(aco_ctx* c, uint16_t* best_tour_host, int64_t* best_len_host) {
    if (aco_status s = usable(c)) return s;
    if (aco_status s = sync_ctx(c, "aco_read_best")) return s;
    hipError_t e = hipSuccess;
    if (best_len_host)
        e = hipMemcpy(best_len_host, c->col.best_len, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && best_tour_host)
        e = hipMemcpy(best_tour_host, c->col.best_tour, ((size_t)c->col.n + 1) * sizeof(uint16_t),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(c, e, "aco_read_best");
    return ACO_OK;
}

aco_status aco_read_tours(aco_ctx* c, uint16_t* tours_host, int64_t* lens_host) {
    if (aco_status s = usable(c)) return s;
    if (aco_status s = sync_ctx(c, "aco_read_tours")) return s;
    const aco::Colony& col = c->col;
    hipError_t e = hipSuccess;
    if (tours_host)
        e = hipMemcpy2D(tours_host, ((size_t)col.n + 1) * sizeof(uint16_t), col.tours,
                        (size_t)col.tp * sizeof(uint16_t), ((size_t)col.n + 1) * sizeof(uint16_t),
                        (size_t)col.m, hipMemcpyDeviceToHost);
    if (e == hipSuccess && lens_host)
        e = hipMemcpy(lens_host, col.lens, (size_t)col.m * sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(c, e, "aco_read_tours");
    return ACO_OK;
}

static aco_status read_matrix(aco_ctx* c, const float* src, float* host, const char* where) {
    if (aco_status s = usable(c)) return s;
    if (!host) return fail(ACO_ERR_INVALID, "host pointer is NULL");
    if (aco_status s = sync_ctx(c, where)) return s;
    const aco::Colony& col = c->col;
    const hipError_t e = hipMemcpy2D(host, (size_t)col.n * sizeof(float), src,
                                     (size_t)col.ld * sizeof(float), (size_t)col.n * sizeof(float),
                                     (size_t)col.n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(c, e, where);
    return ACO_OK;
}

aco_status aco_read_tau(aco_ctx* c, float* tau_host) {
    return read_matrix(c, c ? c->col.tau : nullptr, tau_host, "aco_read_tau");
}

aco_status aco_read_choice(aco_ctx* c, float* choice_host) {
    return read_matrix(c, c ? c->col.choice : nullptr, choice_host, "aco_read_choice");
}

aco_status aco_restore(aco_ctx* c, const float* tau_host, uint32_t iter, int64_t best_len,
                       const uint16_t* best_tour_host) {
    if (aco_status s = usable(c)) return s;
    if (!tau_host) return fail(ACO_ERR_INVALID, "tau_host is NULL");
    if (aco_status s = sync_ctx(c, "aco_restore")) return s;
    const aco::Colony& col = c->col;
    // tau <= 1e18 keeps tau^2 (alpha = 2), every choice value and every
    // product of a choice value with a draw finite
    for (size_t i = 0; i < (size_t)col.n * col.n; ++i)
        if (!(tau_host[i] >= 0.0f && tau_host[i] <= 1e18f))
            return fail(ACO_ERR_INVALID, "tau must be in [0, 1e18]");
    hipError_t e = hipMemcpy2D(col.tau, (size_t)col.ld * sizeof(float), tau_host,
                               (size_t)col.n * sizeof(float), (size_t)col.n * sizeof(float),
                               (size_t)col.n, hipMemcpyHostToDevice);
    const int64_t bl = best_len < 0 ? INT64_MAX : best_len;
    if (e == hipSuccess)
        e = hipMemcpy(col.best_len, &bl, sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && best_tour_host && best_len >= 0)
        e = hipMemcpy(col.best_tour, best_tour_host, ((size_t)col.n + 1) * sizeof(uint16_t),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = aco::launch_refresh_choice(col, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return device_fail(c, e, "aco_restore");
    c->next_iter = iter;
    c->pending = false;
    return ACO_OK;
}

aco_status aco_get_iter(aco_ctx* c, uint32_t* iter) {
    if (aco_status s = usable(c)) return s;
    if (!iter) return fail(ACO_ERR_INVALID, "iter is NULL");
    *iter = c->next_iter;
    return ACO_OK;
}

aco_status aco_sync(aco_ctx* c) {
    if (aco_status s = usable(c)) return s;
    return sync_ctx(c, "aco_sync");
}

void aco_destroy(aco_ctx* c) { delete c; }

aco_status aco_describe(aco_ctx* c, char* buf, size_t len) {
    if (!c) return fail(ACO_ERR_INVALID, "context is NULL");
    if (!buf || len == 0) return fail(ACO_ERR_INVALID, "buffer is NULL");
    const aco::Colony& col = c->col;
    int dev = 0, cus = 0, lds_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    const int pass = 64 * col.tile;
    std::snprintf(buf, len,
                  "construct=workgroup_per_ant waves_per_ant=%d cities_per_lane=%d passes=%d "
                  "blocks=%d ld=%d ants_per_cu=%d cus=%d lds_per_cu=%d "
                  "update_gather_threads=256 atomic=%d nn=%d",
                  col.waves, col.tile, (col.n + pass - 1) / pass, (col.n + 63) / 64, col.ld,
                  aco::construct_occupancy(col), cus, lds_cu, c->has_atomic ? 1 : 0, c->nn.nn);
    return ACO_OK;
}

aco_status aco_test_select_shape(int32_t tile, int32_t waves, int32_t n, int32_t count,
                                 const float* rows_dev, const uint8_t* feasible_dev,
                                 const float* u_dev, int32_t* out_dev, void* hip_stream) {
    if (n < 1 || n > aco::kMaxCities) return fail(ACO_ERR_INVALID, "n must be in [1, 4096]");
    if (!aco::host::shape_supported(tile, waves, n))
        return fail(ACO_ERR_INVALID, "construction shape not supported for this n");
    if (count < 0) return fail(ACO_ERR_INVALID, "count must be >= 0");
    if (count > 0 && (!rows_dev || !feasible_dev || !u_dev || !out_dev))
        return fail(ACO_ERR_INVALID, "NULL device pointer");
    if (((uintptr_t)rows_dev % 16) != 0)
        return fail(ACO_ERR_INVALID, "rows must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const hipError_t e =
        waves == 1 ? aco::launch_test_select(tile, n, count, rows_dev, feasible_dev, u_dev,
                                             out_dev, s)
                   : aco::launch_test_select_split(tile, waves, n, count, rows_dev,
                                                   feasible_dev, u_dev, out_dev, s);
    if (e != hipSuccess) return device_fail(nullptr, e, "aco_test_select");
    return ACO_OK;
}

aco_status aco_test_select(int32_t tile, int32_t n, int32_t count, const float* rows_dev,
                           const uint8_t* feasible_dev, const float* u_dev, int32_t* out_dev,
                           void* hip_stream) {
    if (n >= 1 && n <= aco::kMaxCities && !aco::tile_supported(tile, n))
        return fail(ACO_ERR_INVALID, "tile must be 8 (any n) or 4 (n <= 1024)");
    return aco_test_select_shape(tile, 1, n, count, rows_dev, feasible_dev, u_dev, out_dev,
                                 hip_stream);
}

aco_status aco_probe_copy(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream) {
    if (bytes % 16 != 0) return fail(ACO_ERR_INVALID, "bytes must be a multiple of 16");
    if (bytes && (!dst_dev || !src_dev)) return fail(ACO_ERR_INVALID, "NULL device pointer");
    if (((uintptr_t)dst_dev | (uintptr_t)src_dev) % 16 != 0)
        return fail(ACO_ERR_INVALID, "buffers must be 16-byte aligned");
    const hipError_t e =
        aco::launch_probe_copy(dst_dev, src_dev, bytes, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return device_fail(nullptr, e, "aco_probe_copy");
    return ACO_OK;
}

aco_status aco_probe_read(const void* src_dev, size_t bytes, int32_t reps, float* sink_dev,
                          void* hip_stream) {
    if (bytes % 16 != 0) return fail(ACO_ERR_INVALID, "bytes must be a multiple of 16");
    if (reps < 0) return fail(ACO_ERR_INVALID, "reps must be >= 0");
    if (bytes && (!src_dev || !sink_dev)) return fail(ACO_ERR_INVALID, "NULL device pointer");
    if (((uintptr_t)src_dev % 16) != 0) return fail(ACO_ERR_INVALID, "src must be 16-byte aligned");
    const hipError_t e = aco::launch_probe_read(src_dev, bytes, reps, 4, false, sink_dev,
                                                static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return device_fail(nullptr, e, "aco_probe_read");
    return ACO_OK;
}

aco_status aco_probe_read_shape(const void* src_dev, size_t bytes, int32_t reps,
                                int32_t loads_in_flight, int32_t nontemporal, float* sink_dev,
                                void* hip_stream) {
    if (bytes % 16 != 0) return fail(ACO_ERR_INVALID, "bytes must be a multiple of 16");
    if (reps < 0) return fail(ACO_ERR_INVALID, "reps must be >= 0");
    if (loads_in_flight != 4 && loads_in_flight != 8 && loads_in_flight != 16)
        return fail(ACO_ERR_INVALID, "loads_in_flight must be 4, 8 or 16");
    if (bytes && (!src_dev || !sink_dev)) return fail(ACO_ERR_INVALID, "NULL device pointer");
    if (((uintptr_t)src_dev % 16) != 0) return fail(ACO_ERR_INVALID, "src must be 16-byte aligned");
    const hipError_t e =
        aco::launch_probe_read(src_dev, bytes, reps, loads_in_flight, nontemporal != 0, sink_dev,
                               static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return device_fail(nullptr, e, "aco_probe_read_shape");
    return ACO_OK;
}

aco_status aco_probe_philox(int32_t waves, int32_t steps, uint32_t seed, uint32_t* sink_dev,
                            void* hip_stream) {
    if (waves < 0 || steps < 0) return fail(ACO_ERR_INVALID, "waves and steps must be >= 0");
    if (waves > 0 && !sink_dev) return fail(ACO_ERR_INVALID, "NULL device pointer");
    const hipError_t e = aco::launch_probe_philox(waves, steps, seed, sink_dev,
                                                  static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return device_fail(nullptr, e, "aco_probe_philox");
    return ACO_OK;
}

aco_status aco_probe_rows_shape(const float* mat_dev, int32_t rows, int32_t ld,
                                int32_t row_len, int32_t waves, int32_t steps,
                                int32_t rows_in_flight, float* sink_dev, void* hip_stream) {
    if (rows < 1 || row_len < 1 || row_len > aco::kMaxCities || ld < row_len || (ld % 4) != 0)
        return fail(ACO_ERR_INVALID, "need rows >= 1, 1 <= row_len <= 4096, ld >= row_len, ld % 4 == 0");
    if (waves < 0 || steps < 0) return fail(ACO_ERR_INVALID, "waves and steps must be >= 0");
    if (rows_in_flight != 1 && rows_in_flight != 2)
        return fail(ACO_ERR_INVALID, "rows_in_flight must be 1 or 2");
    if (waves > 0 && (!mat_dev || !sink_dev)) return fail(ACO_ERR_INVALID, "NULL device pointer");
    if (((uintptr_t)mat_dev % 16) != 0) return fail(ACO_ERR_INVALID, "matrix must be 16-byte aligned");
    const hipError_t e =
        aco::launch_probe_rows(mat_dev, rows, ld, row_len, waves, steps, rows_in_flight, sink_dev,
                               static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return device_fail(nullptr, e, "aco_probe_rows");
    return ACO_OK;
}

aco_status aco_probe_rows(const float* mat_dev, int32_t rows, int32_t ld, int32_t row_len,
                          int32_t waves, int32_t steps, float* sink_dev, void* hip_stream) {
    return aco_probe_rows_shape(mat_dev, rows, ld, row_len, waves, steps, 1, sink_dev,
                                hip_stream);
}

}  // extern "C"
