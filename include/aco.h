/*
 * aco.h -- C ABI of libaco, an Ant System (AS) solver for the symmetric
 * Euclidean TSP on AMD Instinct MI355X (gfx950).
 *
 * The library runs the two stages of an AS iteration on the GPU, following
 * Cecilia et al., "Parallelization Strategies for Ant Colony Optimisation on
 * GPUs" (arXiv:1101.2678):
 *   - tour construction (Section II, Eq. 1; GPU design in Section III-A): one
 *     workgroup per ant, cities spread over the lanes, next city drawn by
 *     proportional roulette over choice = tau^alpha * eta^beta (eta = 1/d)
 *     restricted to unvisited cities;
 *   - pheromone update (Section II, Eqs. 2-4; GPU designs in Section III-B):
 *     evaporation tau <- (1 - rho) tau, then every ant k deposits 1/C^k on
 *     each edge of its tour, in either a scatter-to-gather (row owner) or an
 *     atomic-deposit variant; the choice matrix is refreshed in the same pass.
 * Two further construction rules share the update: the nearest-neighbour
 * candidate lists of Section II (aco_construct_nn) and the paper's own
 * data-parallel product-and-argmax selection of Section III-A
 * (aco_construct_product).  Many instances run together through the batch
 * API (aco_batch_*), and a continuous-batching server (aco_server_*) admits
 * solve requests by resident footprint while others run.
 *
 * Conventions for every entry point:
 *   - Nothing throws or aborts across the ABI; every call returns aco_status.
 *   - "host" pointers are ordinary CPU memory, borrowed for the duration of
 *     the call only.  "device" pointers are GPU memory owned by the caller.
 *   - Work is enqueued on the caller's HIP stream (passed as void*, a
 *     hipStream_t; NULL is the default stream).  Calls documented as
 *     asynchronous return before the GPU finishes; the synchronous ones wait
 *     on that stream.  A device error is reported as ACO_ERR_DEVICE by the
 *     call that observes it, after which the context is poisoned and every
 *     later call on it returns ACO_ERR_STATE.
 *   - A context is not thread-safe.  Distinct contexts may run concurrently
 *     on distinct streams.
 *
 * Arithmetic (identical on every path, and bit-exact against the oracle):
 *   - random numbers: Philox4x32-10 with key = seed and counter
 *     (step, ant, iter, 0); word 0 gives the start city ((x0*n) >> 32) at
 *     step 0 and u = (x0 >> 8) * 2^-24 at step s >= 1;
 *   - roulette ("R64"): feasible weights w_j = choice[i][j], blocks of 64
 *     cities scanned by a fixed FP32 prefix tree, block totals scanned by the
 *     same tree; the next city is the lowest feasible j whose prefix exceeds
 *     fl32(u * total), else the highest feasible city;
 *   - heur = fl32(1 / d^beta) (binary64 power and quotient), choice =
 *     fl32(tau^alpha * heur), zero on the diagonal;
 *   - update: tau <- fl32((double)fl32(tau * fl32(1 - rho)) + D) where D is the
 *     binary64 sum of fl32(1 / C^k) over the ants using the edge (exact, so
 *     independent of summation order);
 *   - tau0 = fl32(m / C_nn), C_nn the nearest-neighbour tour length from
 *     city 0 (ties to the lowest index).
 */
#ifndef ACO_H
#define ACO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ACO_OK = 0,
    ACO_ERR_INVALID = 1, /* bad argument; nothing was enqueued */
    ACO_ERR_NOMEM = 2,   /* workspace too small or misaligned */
    ACO_ERR_DEVICE = 3,  /* a HIP call or kernel failed; context poisoned */
    ACO_ERR_STATE = 4    /* call out of order, or context poisoned */
} aco_status;

/* Pheromone update variants (Section III-B); all three give the same bits.
 *   GATHER         scatter-to-gather: one workgroup owns row i, reads the tour
 *                  neighbours of city i in every ant's tour and writes the
 *                  row; no global atomics.
 *   ATOMIC         one thread per city of an ant's tour, deposits combined in
 *                  shared memory (LDS) per row, then one global binary64
 *                  atomic per distinct edge ("atomic instructions + shared
 *                  memory", the paper's fastest update).
 *   ATOMIC_DIRECT  one global binary64 atomic per tour edge ("atomic
 *                  instructions").
 * Both atomic kinds need the atomic part of the workspace. */
typedef enum {
    ACO_UPDATE_GATHER = 0,
    ACO_UPDATE_ATOMIC = 1,
    ACO_UPDATE_ATOMIC_DIRECT = 2
} aco_update_kind;

/* Problem and AS parameters.
 *   n      number of cities, 3 <= n <= 4096
 *   m      number of ants, 1 <= m <= 65535 (the paper uses m = n)
 *   alpha  pheromone exponent, 0, 1 or 2
 *   beta   heuristic exponent, 0 <= beta <= 4
 *   rho    evaporation rate, 0 < rho <= 1 (Eq. 2)
 *   seed   Philox key */
typedef struct {
    int32_t n;
    int32_t m;
    int32_t alpha;
    int32_t beta;
    float rho;
    uint64_t seed;
} aco_params;

typedef struct aco_ctx aco_ctx; /* opaque; host memory owned by the library */

/* Exact number of device bytes aco_init needs for these parameters.
 * with_atomic != 0 also reserves the binary64 deposit matrix that
 * ACO_UPDATE_ATOMIC uses (8 * n * ld bytes, ld = n rounded up to 64).
 * Returns 0 if the parameters are invalid. */
size_t aco_workspace_bytes(const aco_params* p, int32_t with_atomic);

/* Create a context on the current HIP device.
 *   out          receives the context (host)
 *   p            parameters (host)
 *   dist_host    n*n int32 row-major distances (host, borrowed for the call);
 *                must be symmetric with a zero diagonal and d_ij >= 1 off it
 *   d_workspace  device buffer of ws_bytes >= aco_workspace_bytes(p, 0),
 *                256-byte aligned, owned by the caller and never freed by the
 *                library; it holds tau, choice, distances, tours and all
 *                per-iteration state.  If ws_bytes also covers the atomic
 *                size, ACO_UPDATE_ATOMIC is available.
 *   hip_stream   the stream every later call of this context enqueues on;
 *                NULL (the default stream) or a stream created on the current
 *                device by the HIP runtime this library is linked against
 * Uploads the distances, computes C_nn and tau0 on the GPU, fills tau and
 * choice.  Synchronous.  Errors: ACO_ERR_INVALID (parameters, distances, a
 * stream of another device), ACO_ERR_NOMEM (workspace), ACO_ERR_DEVICE (a
 * stream handle the runtime does not know, or a failed HIP call). */
aco_status aco_init(aco_ctx** out, const aco_params* p, const int32_t* dist_host,
                    void* d_workspace, size_t ws_bytes, void* hip_stream);

/* Tour construction for iteration `iter` (Section II, Eq. 1): all m ants
 * build a tour from the current choice matrix; writes tours, lengths C^k and
 * deposits fl32(1/C^k).  One kernel launch.  Asynchronous. */
aco_status aco_construct(aco_ctx* c, uint32_t iter);

/* Best-so-far tour (the shortest of the last construction, lowest ant index
 * among equals, replaces the stored one only if strictly shorter), then the
 * pheromone update (Eqs. 2-4) from those tours and the choice refresh.
 * Asynchronous.  ACO_ERR_STATE if no construction preceded
 * it since the last update; ACO_ERR_INVALID for an atomic kind without the
 * atomic workspace or an unknown kind. */
aco_status aco_update(aco_ctx* c, aco_update_kind kind);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * aco_update(c, ACO_UPDATE_ATOMIC) with the binary64 deposit matrix held in
 * a static device array of the library (8 MiB per GPU, kept until the
 * process ends) instead of the workspace, so the context may have been
 * created with aco_workspace_bytes(p, 0).  Same results, bit for bit, as
 * aco_update(c, ACO_UPDATE_ATOMIC).  Allocates nothing: no hipMalloc, no
 * hipFree, no allocating library call.
 *   Limit: n <= 1024 (n * ld <= 2^20 cells), else ACO_ERR_INVALID and nothing
 *   is enqueued.
 *   The array is cleared on the context's stream at the start of every call.
 *   Every call on one GPU shares it: calls whose work overlaps on one GPU
 *   (contexts on different streams, not ordered by the caller) race and give
 *   wrong tau.
 * Asynchronous.  Other errors as aco_update; ACO_ERR_DEVICE if the array's
 * device address could not be obtained at aco_init. */
aco_status aco_update_atomic_noalloc(aco_ctx* c);

/* Runs `iters` iterations (construct, update) starting at the context's
 * iteration counter, then copies the best-so-far tour (n+1 uint16, host) and
 * its length (host) out.  Synchronous.  Either output pointer may be NULL. */
aco_status aco_solve(aco_ctx* c, uint32_t iters, aco_update_kind kind,
                     uint16_t* best_tour_host, int64_t* best_len_host);

/* ---- the paper's product-and-argmax selection --------------------------- */

/* Construction with the data-parallel selection of Section III-A: at city i
 * every unvisited city j draws its own uniform r_j and the next city is the
 * unvisited j with the largest fl32(choice[i][j] * r_j), lowest j among equal
 * products (visited cities take no part; the tiles' winners compete on the
 * same product, so the tiling cannot change the result).  r_j = (x >> 8) *
 * 2^-24 with x = word (j mod 4) of Philox4x32-10, key = seed, counter
 * (step, ant, iter, 1 + j / 4); the start city is drawn as for aco_construct.
 * This is not a sample of Eq. (1): the win probabilities differ from the
 * proportional ones.  Tours, lengths, deposits and the update are those of
 * aco_construct / aco_update.  Asynchronous. */
aco_status aco_construct_product(aco_ctx* c, uint32_t iter);

/* aco_solve with aco_construct_product in place of aco_construct.
 * Synchronous. */
aco_status aco_solve_product(aco_ctx* c, uint32_t iters, aco_update_kind kind,
                             uint16_t* best_tour_host, int64_t* best_len_host);

/* ---- nearest-neighbour candidate lists --------------------------------- */

/* Construction over candidate lists (Section II: the ant chooses among the
 * nn nearest cities of its current city, and takes the best city by the
 * Eq. (1) value once all of them are visited; nn = 30 in the evaluation of
 * Section IV).  Rule, bit-exact against the oracle: row i's list holds the
 * nn cities j != i with the smallest d_ij, ordered by (d_ij, j); at city i,
 * if some list entry is unvisited, the R64 roulette runs over the list in
 * list order (weights choice[i][j] of the unvisited entries, +0 for the
 * others; one 64-entry block) with the same draw u as full construction;
 * otherwise the next city is the unvisited city with the largest
 * choice[i][j], lowest j among equal values.  Tours, lengths, deposits and
 * the update are those of aco_construct / aco_update. */

/* Device bytes of the candidate tables for n cities and lists of nn
 * (1 <= nn <= min(64, n - 1)); 0 if the arguments are invalid. */
size_t aco_nn_workspace_bytes(int32_t n, int32_t nn);

/* Builds the lists of length nn from the context's distances on the device
 * and keeps them for aco_construct_nn.  d_nn_workspace: device buffer of
 * bytes >= aco_nn_workspace_bytes(n, nn), 256-byte aligned, owned by the
 * caller and kept alive as long as the context uses it (a later attach
 * replaces it).  Asynchronous.  Errors: ACO_ERR_INVALID (nn), ACO_ERR_NOMEM
 * (workspace). */
aco_status aco_nn_attach(aco_ctx* c, int32_t nn, void* d_nn_workspace, size_t bytes);

/* aco_construct with the candidate-list rule: rebuilds the packed candidate
 * table from the current choice matrix, then builds the m tours of
 * iteration `iter`.  Asynchronous.  ACO_ERR_STATE without aco_nn_attach. */
aco_status aco_construct_nn(aco_ctx* c, uint32_t iter);

/* aco_solve with aco_construct_nn in place of aco_construct.  Synchronous. */
aco_status aco_solve_nn(aco_ctx* c, uint32_t iters, aco_update_kind kind,
                        uint16_t* best_tour_host, int64_t* best_len_host);

/* Copies the lists (n*nn uint16, row-major, host) out.  Synchronous. */
aco_status aco_read_nn_lists(aco_ctx* c, uint16_t* lists_host);

/* Copies of the device state into host memory.  Synchronous.
 *   tours: m*(n+1) uint16 of the last construction; lens: m int64 (either may
 *   be NULL); tau, choice: n*n float row-major; best_tour: n+1 uint16. */
aco_status aco_read_tours(aco_ctx* c, uint16_t* tours_host, int64_t* lens_host);
aco_status aco_read_tau(aco_ctx* c, float* tau_host);
aco_status aco_read_choice(aco_ctx* c, float* choice_host);
aco_status aco_read_best(aco_ctx* c, uint16_t* best_tour_host, int64_t* best_len_host);

/* Checkpoint restore: replaces tau with the host copy (n*n row-major, e.g.
 * from aco_read_tau; every value in [0, 1e18], else ACO_ERR_INVALID, which
 * keeps every choice value finite), recomputes choice, and sets the iteration counter and
 * best-so-far length (best tour cleared if best_len < 0).  Because every
 * random number is keyed by (seed, iter, ant, step), a resumed run
 * reproduces the uninterrupted one.  Synchronous. */
aco_status aco_restore(aco_ctx* c, const float* tau_host, uint32_t iter, int64_t best_len,
                       const uint16_t* best_tour_host);

/* Iteration counter used by aco_solve (the next iteration to run). */
aco_status aco_get_iter(aco_ctx* c, uint32_t* iter);

/* Waits for all work of this context's stream. */
aco_status aco_sync(aco_ctx* c);

/* Frees the host context.  Never touches the workspace. */
void aco_destroy(aco_ctx* c);

const char* aco_status_str(aco_status s);

/* Human-readable detail of the last failure on this thread ("" if none). */
const char* aco_last_error(void);

/* Kernel configuration chosen for a context, as "key=value" pairs. */
aco_status aco_describe(aco_ctx* c, char* buf, size_t len);

/* ---- verification and measurement entry points ------------------------ */

/* R64 roulette on `count` independent rows through the same device code the
 * construction kernel uses (Section II, Eq. 1).
 *   tile          cities per lane of the construction tile to use (4 or 8;
 *                 4 only for n <= 1024); the result must not depend on it
 *   rows_dev      count rows of `ld` floats (device), ld = n rounded up to
 *                 64; columns n..ld-1 must be zero
 *   feasible_dev  count*n uint8 (device), non-zero = city may be chosen
 *   u_dev         count floats in [0, 1) (device)
 *   out_dev       count int32 (device): the chosen city, -1 if none feasible
 * Asynchronous on hip_stream. */
aco_status aco_test_select(int32_t tile, int32_t n, int32_t count, const float* rows_dev,
                           const uint8_t* feasible_dev, const float* u_dev, int32_t* out_dev,
                           void* hip_stream);

/* As aco_test_select, through the construction kernel of the given shape:
 * `waves` wavefronts per ant share the row (1, or 2 / 4 where
 * aco_set_shape accepts the shape for n).  The result must not depend on
 * tile or waves.  Asynchronous on hip_stream. */
aco_status aco_test_select_shape(int32_t tile, int32_t waves, int32_t n, int32_t count,
                                 const float* rows_dev, const uint8_t* feasible_dev,
                                 const float* u_dev, int32_t* out_dev, void* hip_stream);

/* The product selection on `count` independent rows through the device code
 * aco_construct_product uses, with the draws given instead of generated.
 *   rows_dev      count rows of ld floats (device), ld = n rounded up to 64,
 *                 columns n..ld-1 zero, 16-byte aligned
 *   feasible_dev  count*n uint8 (device), non-zero = city may be chosen
 *   u_dev         count*n floats (device): the draw of every city of the row
 *   out_dev       count int32 (device): the chosen city, -1 if none feasible
 * Asynchronous on hip_stream. */
aco_status aco_test_product_select(int32_t n, int32_t count, const float* rows_dev,
                                   const uint8_t* feasible_dev, const float* u_dev,
                                   int32_t* out_dev, void* hip_stream);

/* ---- construction shapes ----------------------------------------------- */

/* The construction kernel spreads a choice row over the threads of an ant's
 * workgroup (the paper's city tiling and thread blocks, Section III-A):
 * `cities_per_lane` (4 or 8) consecutive cities per lane per pass of
 * 64 * cities_per_lane cities, and `waves_per_ant` wavefronts per ant that
 * share the passes (wave w takes passes w, w + W, ...).  The shape changes
 * speed only, never results.  Supported shapes:
 *   1 wavefront:  tile 8 for any n; tile 4 for n <= 1024;
 *   2 wavefronts: n <= 1024 with at least 2 passes (tile 8: n >= 513;
 *                 tile 4: n >= 257);
 *   4 wavefronts: tile 4 with 4 passes (769 <= n <= 1024).
 * aco_set_shape sets the shape for instance sizes n_lo..n_hi and fails if
 * any size of the range does not support it; aco_set_tile(lo, hi, t) is
 * aco_set_shape(lo, hi, t, 1).  Contexts created afterwards use the table
 * (batched construction always runs one wavefront per ant and takes only the
 * tile).  The table is process-wide and not thread-safe.  Default: tile 4
 * for n <= 256, 8 above, one wavefront per ant. */
aco_status aco_set_shape(int32_t n_lo, int32_t n_hi, int32_t cities_per_lane,
                         int32_t waves_per_ant);
aco_status aco_set_tile(int32_t n_lo, int32_t n_hi, int32_t cities_per_lane);
int32_t aco_get_tile(int32_t n);
int32_t aco_get_waves(int32_t n);
/* Restores the default table (above).  Same thread-safety as aco_set_shape. */
void aco_reset_tiles(void);

/* The shapes the autotuner times, as (cities per lane, wavefronts per ant),
 * in the order of its ms columns: 0 = (4, 1), 1 = (8, 1), 2 = (8, 2),
 * 3 = (4, 2), 4 = (4, 4). */
#define ACO_NUM_SHAPES 5

/* Autotuner: for each of the `count` strictly increasing instance sizes
 * (3..4096), builds a synthetic uniform instance with m = n on d_workspace
 * (>= aco_workspace_bytes for the largest size with m = n, without the
 * atomic part), times `reps` constructions with every shape that supports
 * the size, and sets the shape table so that bucket i, sizes
 * (sizes[i-1], sizes[i]] (the last bucket up to 4096), uses the fastest;
 * sizes of the bucket that shape does not support get its tile with one
 * wavefront (tile 8 where tile 4 stops).
 *   chosen_tile, chosen_waves  count int32 each: the shape picked per size
 *   ms                         count * ACO_NUM_SHAPES floats, row i for
 *                              sizes[i]: ms per construction, -1 where the
 *                              shape does not support the size
 * Each output may be NULL.  Synchronous; overwrites the workspace. */
aco_status aco_autotune(void* d_workspace, size_t ws_bytes, const int32_t* sizes, int32_t count,
                        int32_t reps, void* hip_stream, int32_t* chosen_tile,
                        int32_t* chosen_waves, float* ms);

/* ---- batches: many independent instances advanced together --------------- */

typedef struct aco_batch aco_batch; /* opaque; host memory owned by the library */

/* Exact device bytes for a batch of `count` instances (params: count
 * entries, host).  Returns 0 if any parameter set is invalid. */
size_t aco_batch_workspace_bytes(int32_t count, const aco_params* params);

/* Creates a batch of `count` independent instances (1..65535): instance q has
 * params[q] and the n_q*n_q distances dist_hosts[q] (host, borrowed).  All
 * state lives in d_workspace (caller-owned, 256-byte aligned, >=
 * aco_batch_workspace_bytes).  Instances are scheduled largest n first.
 * Every instance starts at iteration 0 and computes exactly what a context of
 * its own computes with the gather update.  hip_stream as for aco_init (same
 * errors).  Synchronous. */
aco_status aco_batch_init(aco_batch** out, int32_t count, const aco_params* params,
                          const int32_t* const* dist_hosts, void* d_workspace, size_t ws_bytes,
                          void* hip_stream);

/* Advances every instance by `iters` iterations (construction, best-so-far,
 * gather update): three launches per iteration for the whole batch.  With
 * use_graph != 0 the launches are captured once into a HIP graph (kept for
 * the next call with the same `iters`) and replayed; this needs a
 * non-default stream.  Asynchronous. */
aco_status aco_batch_run(aco_batch* b, uint32_t iters, int32_t use_graph);

/* Launch configuration of a batch's construction.  It changes speed only,
 * never results (the paper's tiling and block-size choices, Section III-A).
 *   wg_per_cu    at most this many construction workgroups (ants) resident
 *                on a compute unit, enforced through the workgroup's LDS
 *                request (the device's LDS per CU / wg_per_cu); 0 = no cap
 *                (registers and LDS of the tour decide).  Each resident ant
 *                keeps one choice row in flight: more of them evict one
 *                another's rows from the L2, fewer leave its latency bare.
 *   tile4_max_n  instances with n <= tile4_max_n use 4 cities per lane and
 *                pass, the others 8 (at most 1024); -1 = the process-wide
 *                tile table (aco_set_tile / aco_autotune).
 * Default after aco_batch_init: tile4_max_n = -1, and wg_per_cu = 16 when
 * the batch has at least 8 * 16 ants per compute unit, else 0. */
typedef struct {
    int32_t wg_per_cu;
    int32_t tile4_max_n;
} aco_batch_config;

/* Sets the launch configuration; waits for the batch's stream and drops a
 * captured graph (the next graph run captures again).  ACO_ERR_INVALID if
 * wg_per_cu is outside [0, 64] or asks for more LDS than one workgroup may
 * hold, or tile4_max_n is outside [-1, 1024].  Synchronous. */
aco_status aco_batch_set_config(aco_batch* b, const aco_batch_config* cfg);
aco_status aco_batch_get_config(aco_batch* b, aco_batch_config* cfg);

/* Autotuner of the batched launch: for each of the `count` candidate
 * configurations (host array), one warm-up iteration and then `iters` timed
 * iterations of the whole batch (eager launches, HIP events on the batch's
 * stream); keeps the fastest configuration.  best_index (host, may be NULL)
 * receives its index, ms_per_iter (count floats, host, may be NULL) every
 * candidate's time per iteration.  Advances every instance by
 * count * (iters + 1) iterations, computed exactly as any other iterations
 * of the batch.  Synchronous. */
aco_status aco_batch_autotune(aco_batch* b, const aco_batch_config* cands, int32_t count,
                              uint32_t iters, int32_t* best_index, float* ms_per_iter);

/* Per-instance reads (q in caller order).  Synchronous. */
aco_status aco_batch_read_best(aco_batch* b, int32_t q, uint16_t* best_tour_host,
                               int64_t* best_len_host);
aco_status aco_batch_read_tours(aco_batch* b, int32_t q, uint16_t* tours_host,
                                int64_t* lens_host);
aco_status aco_batch_read_tau(aco_batch* b, int32_t q, float* tau_host);
aco_status aco_batch_get_iter(aco_batch* b, int32_t q, uint32_t* iter);
aco_status aco_batch_sync(aco_batch* b);
/* Waits for the batch's stream if a captured graph exists, releases the
 * graph and the host state; never touches the workspace. */
void aco_batch_destroy(aco_batch* b);

/* Streams `bytes` (multiple of 16) from src_dev to dst_dev with 16-byte loads
 * and stores: a plain copy kernel of known traffic, used to calibrate
 * hardware byte counters and to measure achievable bandwidth.  Async. */
aco_status aco_probe_copy(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream);

/* Reads `bytes` (multiple of 16) of src_dev `reps` times in all and writes
 * one float per workgroup to sink_dev (>= 4096 floats, device): the
 * streaming read bandwidth of a footprint.  Each of the eight XCDs walks the
 * whole buffer in 16 KB chunks (reps / 8 times), so every XCD's L2 sees the
 * full footprint, as it does in tour construction: a buffer larger than the
 * L2 (4 MB per XCD) is served by the Infinity Cache (256 MB) or, beyond that,
 * by HBM.  Algorithmic bytes: bytes * reps.  Asynchronous. */
aco_status aco_probe_read(const void* src_dev, size_t bytes, int32_t reps, float* sink_dev,
                          void* hip_stream);

/* aco_probe_read with a chosen load shape: loads_in_flight 16-byte loads per
 * thread issued before any is used (4, 8 or 16; aco_probe_read uses 4), and
 * nontemporal != 0 for loads that keep nothing in the caches.  The streaming
 * ceiling of a footprint is the best rate over the shapes.  Async. */
aco_status aco_probe_read_shape(const void* src_dev, size_t bytes, int32_t reps,
                                int32_t loads_in_flight, int32_t nontemporal, float* sink_dev,
                                void* hip_stream);

/* ---- serving: continuous batching of independent solves ------------------ */

typedef struct aco_server aco_server; /* opaque; host memory owned by the library */

/* Bytes the server reserves at the head of its pool for the tables of the
 * running sets: per size class, max_slots colonies, max_ants ant entries and
 * max_rows row entries.  0 if an argument is out of range. */
size_t aco_server_table_bytes(int32_t max_slots, int32_t max_ants, int32_t max_rows,
                              int32_t num_classes);

/* Creates a server over a caller-owned device pool (256-byte aligned,
 * >= aco_server_table_bytes); the rest of the pool holds request
 * workspaces.  Requests are sorted into num_classes (1..8) size classes by
 * n: class c takes n <= class_max_n[c] (increasing; the last class also
 * takes anything larger).  Each class ticks on a stream of the server's own,
 * independently of the others; request initialisation runs on another.  At
 * most max_slots requests are held at once, and the requests of one class
 * never exceed max_ants ants or max_rows rows in total. */
aco_status aco_server_create(aco_server** out, void* d_pool, size_t pool_bytes, int32_t max_slots,
                             int32_t max_ants, int32_t max_rows, int32_t num_classes,
                             const int32_t* class_max_n);

/* Admission: a request for `iters` iterations of instance (p, dist_host) is
 * admitted if a slot is free, the running set stays within max_ants/max_rows
 * (else ACO_ERR_STATE) and the pool has a free block of
 * aco_workspace_bytes(p, 0) bytes (else ACO_ERR_NOMEM); nothing changes on a
 * refusal.  On success *slot_out receives the slot; the distances are
 * uploaded and the colony initialised asynchronously, and the request joins
 * the running set at the first tick after that.  dist_host must stay valid
 * until aco_server_step has been called once more. */
aco_status aco_server_submit(aco_server* s, const aco_params* p, const int32_t* dist_host,
                             uint32_t iters, int64_t request_id, int32_t* slot_out);

/* Progress without blocking: completes the ticks that have finished (a
 * request whose iterations are all done becomes finished), lets requests
 * whose initialisation has finished join their class, and starts the next
 * tick of every idle class that has running requests.  A tick advances each
 * running request of the class by one iteration (Section II: construction,
 * best-so-far, update) in three launches.  *running_out (may be NULL)
 * receives the number of requests in ticks now in flight. */
aco_status aco_server_step(aco_server* s, int32_t* running_out);

/* Reports (up to max) finished requests not reported before: their slots
 * and request ids.  Does not block. */
aco_status aco_server_collect(aco_server* s, int32_t* slots_out, int64_t* ids_out, int32_t max,
                              int32_t* count_out);

/* Result of a finished request (best tour n+1 uint16, best length; host),
 * its final tau (n*n floats, host), and release of its slot and memory. */
aco_status aco_server_result(aco_server* s, int32_t slot, uint16_t* best_tour_host,
                             int64_t* best_len_host);
aco_status aco_server_read_tau(aco_server* s, int32_t slot, float* tau_host);
aco_status aco_server_release(aco_server* s, int32_t slot);

/* Occupancy: requests running, initialising and finished-but-held, free
 * pool bytes, the largest free block, ticks so far.  Any pointer may be
 * NULL. */
aco_status aco_server_stats(aco_server* s, int32_t* running, int32_t* initialising,
                            int32_t* finished, size_t* free_bytes, size_t* largest_free_block,
                            uint64_t* ticks);
void aco_server_destroy(aco_server* s);

/* Philox throughput probe (measurement of the product rule's compute
 * ceiling): `waves` wavefronts each compute ten Philox4x32-10 blocks per lane
 * per step, exactly as aco_construct_product draws a 2400-city row, for
 * `steps` steps, with no memory traffic besides writing waves * 64 uint32
 * to sink_dev (device).  Asynchronous on hip_stream. */
aco_status aco_probe_philox(int32_t waves, int32_t steps, uint32_t seed, uint32_t* sink_dev,
                            void* hip_stream);

/* Random-row read probe: the access pattern of tour construction without its
 * arithmetic.  `waves` one-wavefront workgroups each read `steps` whole rows
 * of `row_len` floats from a rows x ld float matrix (device), the row of each
 * step a hash of (workgroup, step).  Algorithmic bytes: 4 * row_len * waves *
 * steps.  sink_dev: >= waves floats (device).  ld % 4 == 0, row_len <= 4096.
 * Asynchronous. */
aco_status aco_probe_rows(const float* mat_dev, int32_t rows, int32_t ld, int32_t row_len,
                          int32_t waves, int32_t steps, float* sink_dev, void* hip_stream);
/* As aco_probe_rows with `rows_in_flight` (1 or 2) steps' rows loaded by a
 * wavefront before any of them is used.  Asynchronous. */
aco_status aco_probe_rows_shape(const float* mat_dev, int32_t rows, int32_t ld,
                                int32_t row_len, int32_t waves, int32_t steps,
                                int32_t rows_in_flight, float* sink_dev, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* ACO_H */
