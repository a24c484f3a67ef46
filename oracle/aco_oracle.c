/*
 * aco_oracle.c -- serial CPU oracle for the Ant System on the symmetric TSP.
 *
 * TEST INFRASTRUCTURE ONLY (see aco_oracle.h).  Plain C99, one thread.
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared.
 */
#include "aco_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10.  Salmon, Moraes, Dror and Shaw, "Parallel random numbers:  */
/* as easy as 1, 2, 3", SC'11, Section 3.3: ten rounds of                    */
/*   (L0, R0, L1, R1) -> (hi(M1*R1) ^ L0 ^ k0, lo(M1*R1), hi(M0*R0) ^ L1 ^ k1,  */
/*   lo(M0*R0)) with the counter read as (R0, L0, R1, L1) = (c0, c1, c2, c3), */
/* and the key bumped by the Weyl constants between rounds.                 */
/* ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u /* multiplies counter word 0 */
#define PHILOX_MUL_B 0xCD9E8D57u /* multiplies counter word 2 */
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)c0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

uint32_t oracle_draw(uint64_t seed, uint32_t iter, uint32_t ant, uint32_t step) {
    uint32_t ctr[4] = {step, ant, iter, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[0];
}

float oracle_uniform(uint32_t x0) {
    /* 24 random bits scaled by 2^-24: every value is exact in binary32. */
    return (float)(x0 >> 8) * (1.0f / 16777216.0f);
}

int32_t oracle_start_city(uint32_t x0, int32_t n) {
    return (int32_t)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Heuristic and choice information (Eq. 1, Section III-A "Choice kernel"). */
/* ------------------------------------------------------------------------ */
float oracle_heur(int32_t d, int32_t beta) {
    if (d == 0) return 0.0f; /* diagonal: never a candidate */
    double p = 1.0;
    for (int32_t b = 0; b < beta; ++b) p = p * (double)d;
    return (float)(1.0 / p);
}

static float tau_pow(float t, int32_t alpha) {
    if (alpha == 0) return 1.0f;
    if (alpha == 1) return t;
    return t * t; /* alpha == 2 */
}

void oracle_choice(int32_t n, const float* tau, const int32_t* dist, int32_t alpha,
                   int32_t beta, float* choice) {
    for (int64_t c = 0; c < (int64_t)n * n; ++c) {
        float h = oracle_heur(dist[c], beta);
        choice[c] = tau_pow(tau[c], alpha) * h;
    }
}

/* ------------------------------------------------------------------------ */
/* Initialisation: tau0 = m / C_nn.                                          */
/* ------------------------------------------------------------------------ */
int64_t oracle_nn_tour_length(int32_t n, const int32_t* dist) {
    uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
    if (!seen) return -1;
    int32_t cur = 0;
    seen[0] = 1;
    int64_t len = 0;
    for (int32_t step = 1; step < n; ++step) {
        int32_t best = -1;
        for (int32_t j = 0; j < n; ++j) {
            if (seen[j]) continue;
            if (best < 0 || dist[(int64_t)cur * n + j] < dist[(int64_t)cur * n + best]) best = j;
        }
        len += dist[(int64_t)cur * n + best];
        seen[best] = 1;
        cur = best;
    }
    len += dist[(int64_t)cur * n + 0];
    free(seen);
    return len;
}

void oracle_init(int32_t n, int32_t m, const int32_t* dist, int32_t alpha, int32_t beta,
                 float* tau, float* choice, float* tau0_out) {
    int64_t cnn = oracle_nn_tour_length(n, dist);
    float tau0 = (float)((double)m / (double)cnn);
    for (int64_t c = 0; c < (int64_t)n * n; ++c) tau[c] = tau0;
    oracle_choice(n, tau, dist, alpha, beta, choice);
    if (tau0_out) *tau0_out = tau0;
}

/* ------------------------------------------------------------------------ */
/* S64 and the R64 roulette.                                                 */
/* ------------------------------------------------------------------------ */
void oracle_s64(const float in[64], float out[64]) {
    float a[64], b[64];
    memcpy(a, in, sizeof a);
    /* Stage A: simultaneous shifted adds inside each 16-entry row. */
    for (int shift = 1; shift <= 8; shift *= 2) {
        for (int t = 0; t < 64; ++t) {
            int pos = t % 16;
            float left = (pos >= shift) ? a[t - shift] : 0.0f;
            b[t] = a[t] + left;
        }
        memcpy(a, b, sizeof a);
    }
    /* Stage B: carry row totals forward. */
    float r0 = a[15], r1 = a[31], r2 = a[47];
    float x = r1 + r0;
    for (int t = 0; t < 64; ++t) {
        int row = t / 16;
        if (row == 0) out[t] = a[t];
        else if (row == 1) out[t] = a[t] + r0;
        else if (row == 2) out[t] = a[t] + x;
        else out[t] = (a[t] + r2) + x;
    }
}

int32_t oracle_r64_select(int32_t n, const float* row, const uint8_t* feasible, float u) {
    if (n < 1 || n > 4096) return -1;
    int32_t nb = (n + 63) / 64;
    /* per-block weights and scans */
    float* s = (float*)malloc(sizeof(float) * 64 * (size_t)nb);
    if (!s) return -1;
    float totals[64];
    for (int b = 0; b < 64; ++b) totals[b] = 0.0f;
    for (int32_t b = 0; b < nb; ++b) {
        float w[64];
        for (int t = 0; t < 64; ++t) {
            int32_t j = 64 * b + t;
            w[t] = (j < n && feasible[j]) ? row[j] : 0.0f;
        }
        oracle_s64(w, s + 64 * b);
        totals[b] = s[64 * b + 63];
    }
    float inc[64];
    oracle_s64(totals, inc);
    float total = inc[nb - 1];
    float target = u * total;
    int32_t pick = -1, last_feasible = -1;
    for (int32_t j = 0; j < n; ++j) {
        if (!feasible[j]) continue;
        last_feasible = j;
        int32_t b = j / 64;
        float e = (b == 0) ? 0.0f : inc[b - 1];
        float p = e + s[j];
        if (p > target) {
            pick = j;
            break;
        }
    }
    free(s);
    if (pick < 0) {
        /* no prefix exceeds the target: the highest feasible city */
        for (int32_t j = n - 1; j >= 0; --j)
            if (feasible[j]) return j;
        return -1;
    }
    (void)last_feasible;
    return pick;
}

void oracle_r64_select_batch(int32_t n, int32_t count, const float* rows,
                             const uint8_t* feasible, const float* u, int32_t* out) {
    for (int32_t q = 0; q < count; ++q)
        out[q] = oracle_r64_select(n, rows + (int64_t)q * n, feasible + (int64_t)q * n, u[q]);
}

/* ------------------------------------------------------------------------ */
/* Tour construction (Section II, random proportional rule).                 */
/* ------------------------------------------------------------------------ */
int64_t oracle_construct_ant(int32_t n, const float* choice, const int32_t* dist,
                             uint64_t seed, uint32_t iter, uint32_t ant, uint16_t* tour) {
    uint8_t* feasible = (uint8_t*)malloc((size_t)n);
    if (!feasible) return -1;
    memset(feasible, 1, (size_t)n);
    int32_t cur = oracle_start_city(oracle_draw(seed, iter, ant, 0), n);
    tour[0] = (uint16_t)cur;
    feasible[cur] = 0;
    int64_t len = 0;
    for (int32_t step = 1; step < n; ++step) {
        float u = oracle_uniform(oracle_draw(seed, iter, ant, (uint32_t)step));
        int32_t next = oracle_r64_select(n, choice + (int64_t)cur * n, feasible, u);
        tour[step] = (uint16_t)next;
        feasible[next] = 0;
        len += dist[(int64_t)cur * n + next];
        cur = next;
    }
    tour[n] = tour[0];
    len += dist[(int64_t)cur * n + tour[0]];
    free(feasible);
    return len;
}

void oracle_nn_lists(int32_t n, const int32_t* dist, int32_t nn, uint16_t* out) {
    uint8_t* taken = (uint8_t*)malloc((size_t)n);
    if (!taken) return;
    for (int32_t i = 0; i < n; ++i) {
        memset(taken, 0, (size_t)n);
        taken[i] = 1;
        for (int32_t r = 0; r < nn; ++r) {
            int32_t best = -1;
            for (int32_t j = 0; j < n; ++j) {
                if (taken[j]) continue;
                if (best < 0 || dist[(int64_t)i * n + j] < dist[(int64_t)i * n + best]) best = j;
            }
            out[(int64_t)i * nn + r] = (uint16_t)best;
            taken[best] = 1;
        }
    }
    free(taken);
}

int64_t oracle_construct_ant_nn(int32_t n, const float* choice, const int32_t* dist,
                                const uint16_t* nnl, int32_t nn, uint64_t seed, uint32_t iter,
                                uint32_t ant, uint16_t* tour) {
    uint8_t* feasible = (uint8_t*)malloc((size_t)n);
    float* cand_w = (float*)malloc(sizeof(float) * (size_t)nn);
    uint8_t* cand_f = (uint8_t*)malloc((size_t)nn);
    if (!feasible || !cand_w || !cand_f) {
        free(feasible);
        free(cand_w);
        free(cand_f);
        return -1;
    }
    memset(feasible, 1, (size_t)n);
    int32_t cur = oracle_start_city(oracle_draw(seed, iter, ant, 0), n);
    tour[0] = (uint16_t)cur;
    feasible[cur] = 0;
    int64_t len = 0;
    for (int32_t step = 1; step < n; ++step) {
        float u = oracle_uniform(oracle_draw(seed, iter, ant, (uint32_t)step));
        const uint16_t* list = nnl + (int64_t)cur * nn;
        int any = 0;
        for (int32_t r = 0; r < nn; ++r) {
            cand_w[r] = choice[(int64_t)cur * n + list[r]];
            cand_f[r] = feasible[list[r]];
            any |= cand_f[r];
        }
        int32_t next;
        if (any) {
            next = list[oracle_r64_select(nn, cand_w, cand_f, u)];
        } else {
            next = -1;
            for (int32_t j = 0; j < n; ++j) {
                if (!feasible[j]) continue;
                if (next < 0 || choice[(int64_t)cur * n + j] > choice[(int64_t)cur * n + next])
                    next = j;
            }
        }
        tour[step] = (uint16_t)next;
        feasible[next] = 0;
        len += dist[(int64_t)cur * n + next];
        cur = next;
    }
    tour[n] = tour[0];
    len += dist[(int64_t)cur * n + tour[0]];
    free(feasible);
    free(cand_w);
    free(cand_f);
    return len;
}

float oracle_product_uniform(uint64_t seed, uint32_t iter, uint32_t ant, uint32_t step,
                             int32_t j) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint32_t ctr[4] = {step, ant, iter, 1u + (uint32_t)j / 4u};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return oracle_uniform(out[j % 4]);
}

int32_t oracle_product_select(int32_t n, const float* row, const uint8_t* feasible,
                              const float* r) {
    int32_t best = -1;
    float best_p = 0.0f;
    for (int32_t j = 0; j < n; ++j) {
        if (!feasible[j]) continue;
        const float p = row[j] * r[j];
        if (best < 0 || p > best_p) {
            best = j;
            best_p = p;
        }
    }
    return best;
}

void oracle_product_select_batch(int32_t count, int32_t n, const float* rows,
                                 const uint8_t* feasible, const float* r, int32_t* out) {
    for (int32_t q = 0; q < count; ++q)
        out[q] = oracle_product_select(n, rows + (int64_t)q * n, feasible + (int64_t)q * n,
                                       r + (int64_t)q * n);
}

int64_t oracle_construct_ant_product(int32_t n, const float* choice, const int32_t* dist,
                                     uint64_t seed, uint32_t iter, uint32_t ant,
                                     uint16_t* tour) {
    uint8_t* feasible = (uint8_t*)malloc((size_t)n);
    float* r = (float*)malloc(sizeof(float) * (size_t)n);
    if (!feasible || !r) {
        free(feasible);
        free(r);
        return -1;
    }
    memset(feasible, 1, (size_t)n);
    int32_t cur = oracle_start_city(oracle_draw(seed, iter, ant, 0), n);
    tour[0] = (uint16_t)cur;
    feasible[cur] = 0;
    int64_t len = 0;
    for (int32_t step = 1; step < n; ++step) {
        for (int32_t j = 0; j < n; ++j) r[j] = oracle_product_uniform(seed, iter, ant, (uint32_t)step, j);
        const int32_t next = oracle_product_select(n, choice + (int64_t)cur * n, feasible, r);
        tour[step] = (uint16_t)next;
        feasible[next] = 0;
        len += dist[(int64_t)cur * n + next];
        cur = next;
    }
    tour[n] = tour[0];
    len += dist[(int64_t)cur * n + tour[0]];
    free(feasible);
    free(r);
    return len;
}

void oracle_construct(int32_t n, int32_t m, const float* choice, const int32_t* dist,
                      uint64_t seed, uint32_t iter, uint16_t* tours, int64_t* lens) {
    for (int32_t k = 0; k < m; ++k)
        lens[k] = oracle_construct_ant(n, choice, dist, seed, iter, (uint32_t)k,
                                       tours + (int64_t)k * (n + 1));
}

/* ------------------------------------------------------------------------ */
/* Pheromone update (Eqs. 2-4).                                              */
/* ------------------------------------------------------------------------ */
float oracle_deposit_amount(int64_t len) { return (float)(1.0 / (double)len); }

int32_t oracle_deposit(int32_t n, int32_t m, const uint16_t* tours, const int64_t* lens,
                       double* D) {
    memset(D, 0, sizeof(double) * (size_t)n * (size_t)n);
    /* Exactness of the binary64 sum: every deposit is a binary32 value, so a
     * multiple of 2^(e_min - 24) where 2^(e_min-1) <= smallest deposit.  No
     * cell receives more than m deposits, each below 2^e_max, so every
     * partial sum is an integer multiple of 2^(e_min-24) below
     * m * 2^(e_max - e_min + 24) units; it is exact when that is <= 2^53. */
    int e_min = 1 << 30, e_max = -(1 << 30);
    for (int32_t k = 0; k < m; ++k) {
        int e;
        frexp((double)oracle_deposit_amount(lens[k]), &e);
        if (e < e_min) e_min = e;
        if (e > e_max) e_max = e;
    }
    int count_bits = 0;
    while ((1LL << count_bits) < (long long)m) ++count_bits;
    int32_t status = (count_bits + (e_max - e_min) + 24 <= 53) ? ORACLE_OK : ORACLE_ERR_INEXACT;
    for (int32_t k = 0; k < m; ++k) {
        double dep = (double)oracle_deposit_amount(lens[k]);
        const uint16_t* t = tours + (int64_t)k * (n + 1);
        for (int32_t s = 0; s < n; ++s) {
            int32_t i = t[s], j = t[s + 1];
            D[(int64_t)i * n + j] += dep;
            D[(int64_t)j * n + i] += dep;
        }
    }
    return status;
}

int32_t oracle_update(int32_t n, int32_t m, float rho, const uint16_t* tours,
                      const int64_t* lens, const int32_t* dist, int32_t alpha,
                      int32_t beta, float* tau, float* choice) {
    double* D = (double*)malloc(sizeof(double) * (size_t)n * (size_t)n);
    if (!D) return ORACLE_ERR_NOMEM;
    int32_t status = oracle_deposit(n, m, tours, lens, D);
    float keep = (float)(1.0 - (double)rho);
    for (int64_t c = 0; c < (int64_t)n * n; ++c) {
        float evaporated = tau[c] * keep;                 /* Eq. 2 */
        tau[c] = (float)((double)evaporated + D[c]);      /* Eq. 3 */
    }
    free(D);
    oracle_choice(n, tau, dist, alpha, beta, choice);
    return status;
}

int32_t oracle_best_of(int32_t m, const int64_t* lens, int64_t* best_len) {
    int32_t who = -1;
    for (int32_t k = 0; k < m; ++k) {
        if (lens[k] < *best_len) {
            *best_len = lens[k];
            who = k;
        }
    }
    return who;
}
