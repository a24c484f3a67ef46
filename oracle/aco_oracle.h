/*
 * aco_oracle.h -- serial CPU oracle for the Ant System (AS) on the symmetric
 * Euclidean TSP (Cecilia et al., "Parallelization Strategies for Ant Colony
 * Optimisation on GPUs", arXiv:1101.2678).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant with the HIP
 * path, and it never takes an input produced by the HIP path.
 *
 * Every function is the plain, slow definition: no blocking, no fusion, no
 * reordering beyond what the cited passage states.  Floating point follows
 * IEEE binary32/binary64 round-to-nearest-even; build with
 * -ffp-contract=off and without -ffast-math.
 *
 * Layouts: every n x n matrix is dense row-major (element (i, j) at i*n + j).
 * Tours are m rows of n+1 uint16 city indices, tour[n] == tour[0].
 *
 * Readings of the paper where its text leaves a choice open:
 *   - random numbers: Philox4x32-10, key = seed, counter = (step, ant, iter, 0),
 *     word 0 only; u = (x0 >> 8) * 2^-24; start city = (x0 * n) >> 32;
 *   - the proportional rule of Eq. (1) is sampled by the "R64" roulette: a
 *     fixed-order 64-wide blocked FP32 prefix scan (see oracle_s64 and
 *     oracle_r64_select);
 *   - pheromone deposits (Eqs. 3-4) are summed in binary64 from 0.0 and added
 *     to the evaporated binary32 value with one rounding;
 *   - tau0 = m / C_nn with C_nn the nearest-neighbour tour length from city 0;
 *   - Q = 1 (deposit 1/C^k), evaporation on all n^2 cells.
 *
 * Every function below is pinned by tests/test_oracle_pins.py against
 * something other than itself: a third-party Philox engine (run, not
 * copied), exact rational arithmetic, closed forms, brute force on tiny
 * instances, invariants of the update, and chi-square tests of the sampled
 * selection probabilities.  tests/test_oracle_mutants.py makes plausible
 * mistakes in a copy of aco_oracle.c and checks that the pins catch each
 * one.  No function here is "parity unpinned".
 */
#ifndef ACO_ORACLE_H
#define ACO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by the oracle entry points that can fail. */
#define ORACLE_OK 0
#define ORACLE_ERR_ARG 1      /* invalid argument                              */
#define ORACLE_ERR_INEXACT 2  /* binary64 deposit sum could be inexact (C11)   */
#define ORACLE_ERR_NOMEM 3

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11).
 * ctr[4] and key[2] in, out[4] out. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Word x0 of Philox4x32-10 with key (lo32(seed), hi32(seed)) and counter
 * (step, ant, iter, 0).  Step 0 places the ant, step s >= 1 draws its s-th
 * roulette number. */
uint32_t oracle_draw(uint64_t seed, uint32_t iter, uint32_t ant, uint32_t step);

/* u = (x0 >> 8) * 2^-24, exact in binary32, in [0, 1 - 2^-24]. */
float oracle_uniform(uint32_t x0);

/* Random initial placement (Section II): (x0 * n) >> 32. */
int32_t oracle_start_city(uint32_t x0, int32_t n);

/* heur = fl32(1 / d^beta) with d^beta by left-to-right binary64 products;
 * heur(0) = 0 (the diagonal).  Eq. (1), eta = 1/d. */
float oracle_heur(int32_t d, int32_t beta);

/* choice_ij = fl32(tau_ij^alpha * heur_ij), tau^0 = 1, tau^2 = fl32(tau*tau).
 * Eq. (1) numerator, precomputed once per iteration (Section III-A). */
void oracle_choice(int32_t n, const float* tau, const int32_t* dist,
                   int32_t alpha, int32_t beta, float* choice);

/* Nearest-neighbour tour from city 0 (ties -> lowest index), closing edge
 * included.  Returns C_nn. */
int64_t oracle_nn_tour_length(int32_t n, const int32_t* dist);

/* tau0 = fl32(m / C_nn) written to all n*n cells, then choice from tau. */
void oracle_init(int32_t n, int32_t m, const int32_t* dist, int32_t alpha,
                 int32_t beta, float* tau, float* choice, float* tau0_out);

/* S64: the fixed 64-wide FP32 prefix-sum tree used by the roulette.
 * Stage A: within each 16-entry row, shifted adds by 1, 2, 4, 8 (entries
 * before the row start contribute +0).  Stage B: with R0, R1, R2 the stage-A
 * values at positions 15, 31, 47 and X = R1 + R0: row 1 adds R0, row 2 adds
 * X, row 3 adds R2 and then X. */
void oracle_s64(const float in[64], float out[64]);

/* R64 roulette over one row (Eq. 1 probabilities):
 *   w_j = feasible[j] ? row[j] : +0 (j < n), +0 for padding up to 64*nb;
 *   s_b = S64(block b), T_b = s_b[63], I = S64(T_0..T_{nb-1}, zero padded);
 *   E_0 = +0, E_b = I[b-1], total = I[nb-1], P_j = fl32(E_b + s_b[j mod 64]);
 *   target = fl32(u * total);
 *   j* = min feasible j with P_j > target, else max feasible j.
 * Returns j*, or -1 if no city is feasible.  n <= 4096. */
int32_t oracle_r64_select(int32_t n, const float* row, const uint8_t* feasible, float u);

/* oracle_r64_select on `count` rows (row q at rows + q*n, feasibility at
 * feasible + q*n), one after the other. */
void oracle_r64_select_batch(int32_t n, int32_t count, const float* rows,
                             const uint8_t* feasible, const float* u, int32_t* out);

/* One ant's tour (Section II): placement, then n-1 roulette steps over the
 * choice row of the current city with the visited cities masked out.
 * tour gets n+1 entries; returns the tour length C^k (int64). */
int64_t oracle_construct_ant(int32_t n, const float* choice, const int32_t* dist,
                             uint64_t seed, uint32_t iter, uint32_t ant, uint16_t* tour);

/* All m ants of one iteration.  tours: m*(n+1), lens: m. */
void oracle_construct(int32_t n, int32_t m, const float* choice, const int32_t* dist,
                      uint64_t seed, uint32_t iter, uint16_t* tours, int64_t* lens);

/* Nearest-neighbour lists (Section II, the nn-list variant of construction):
 * row i holds the nn cities j != i with the smallest d_ij, ordered by
 * (d_ij, j).  out: n*nn uint16.  1 <= nn <= n-1. */
void oracle_nn_lists(int32_t n, const int32_t* dist, int32_t nn, uint16_t* out);

/* One ant's tour with nn-list construction: at city i the candidates are the
 * unvisited entries of row i's list, in list order, weighted by
 * choice[i][.]; if any candidate is unvisited the next city is drawn by the
 * R64 roulette over the candidate vector (oracle_r64_select on the nn list
 * entries, same Philox draw as full construction); otherwise it is the
 * unvisited city with the largest choice value (lowest index among equal
 * values).  Returns C^k. */
int64_t oracle_construct_ant_nn(int32_t n, const float* choice, const int32_t* dist,
                                const uint16_t* nnl, int32_t nn, uint64_t seed, uint32_t iter,
                                uint32_t ant, uint16_t* tour);

/* The paper's data-parallel selection (Section III-A): every city j draws its
 * own uniform r_j, the product choice[i][j] * r_j * tabu_j is formed, and the
 * reduction returns the largest.  Reading: visited cities are excluded (not
 * multiplied by 0, which would let them tie at 0), the product is fl32, ties
 * go to the lowest j, and the per-tile winners compete on the same product,
 * so tiling cannot change the result.
 *
 * r_j = (x >> 8) * 2^-24 with x = word (j mod 4) of Philox4x32-10 at counter
 * (step, ant, iter, 1 + j / 4): one Philox block serves four cities, and the
 * counters never meet those of oracle_draw (last word 0). */
float oracle_product_uniform(uint64_t seed, uint32_t iter, uint32_t ant, uint32_t step,
                             int32_t j);

/* argmax over feasible j of fl32(row[j] * r[j]), lowest j among equal
 * products; -1 if no city is feasible. */
int32_t oracle_product_select(int32_t n, const float* row, const uint8_t* feasible,
                              const float* r);

/* count independent selections: rows count*n, feasible count*n, r count*n. */
void oracle_product_select_batch(int32_t count, int32_t n, const float* rows,
                                 const uint8_t* feasible, const float* r, int32_t* out);

/* One ant's tour with the product rule; placement as oracle_construct_ant. */
int64_t oracle_construct_ant_product(int32_t n, const float* choice, const int32_t* dist,
                                     uint64_t seed, uint32_t iter, uint32_t ant,
                                     uint16_t* tour);

/* dep_k = fl32(1 / C^k), Eq. (4) with Q = 1. */
float oracle_deposit_amount(int64_t len);

/* D_ij = sum over ants whose tour holds edge {i,j} of dep_k, both (i,j) and
 * (j,i), summed in binary64 from 0.0 (Eqs. 3-4).  D: n*n doubles (written).
 * Returns ORACLE_ERR_INEXACT if the exactness condition of the binary64 sum
 * fails (then D is still written). */
int32_t oracle_deposit(int32_t n, int32_t m, const uint16_t* tours, const int64_t* lens,
                       double* D);

/* Pheromone update (Section II, Eqs. 2-4): e = fl32(1 - rho);
 * tau_ij <- fl32((double)fl32(tau_ij * e) + D_ij) on all n^2 cells, then the
 * choice matrix is recomputed from the new tau. */
int32_t oracle_update(int32_t n, int32_t m, float rho, const uint16_t* tours,
                      const int64_t* lens, const int32_t* dist, int32_t alpha,
                      int32_t beta, float* tau, float* choice);

/* Best-so-far rule: the first ant (in ant order) with a strictly shorter
 * length than *best_len replaces it.  Returns the ant index or -1. */
int32_t oracle_best_of(int32_t m, const int64_t* lens, int64_t* best_len);

#ifdef __cplusplus
}
#endif
#endif
