"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case copies ``oracle/aco_oracle.c``, makes one plausible mistake in
the copy (a wrong constant, index, comparison, operand order or a dropped
term), builds it into a library of its own and runs the pins of
``test_oracle_pins.py`` that guard that part against it.  At least one of
them must fail.  The unmodified copy, built the same way, must pass every
pin used here.  The oracle itself is never modified.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "aco_oracle.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "aco_oracle.h")

R64_CONSTRUCT_START = (
    "    tour[0] = (uint16_t)cur;\n    feasible[cur] = 0;\n    int64_t len = 0;\n"
    "    for (int32_t step = 1; step < n; ++step) {\n"
    "        float u = oracle_uniform(oracle_draw(seed, iter, ant, (uint32_t)step));\n"
    "        int32_t next")

# name: (text in the oracle, replacement, pins that must catch it)
MUTANTS = {
    "philox_weyl_constant": (
        "k1 += PHILOX_WEYL_B;", "k1 += PHILOX_WEYL_A;",
        [("test_philox_matches_rocrand", "tpf")]),
    "philox_wrong_word": (
        "uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;", "uint32_t n0 = (uint32_t)(pb >> 32) ^ c3 ^ k0;",
        [("test_philox_matches_rocrand", "tpf")]),
    "draw_counter_swapped": (
        "uint32_t ctr[4] = {step, ant, iter, 0u};", "uint32_t ctr[4] = {ant, step, iter, 0u};",
        [("test_draw_keying", None)]),
    "uniform_23_bits": (
        "return (float)(x0 >> 8) * (1.0f / 16777216.0f);",
        "return (float)(x0 >> 9) * (1.0f / 8388608.0f);",
        [("test_uniform_grid_and_range", None)]),
    "start_city_never_last": (
        "return (int32_t)(((uint64_t)x0 * (uint64_t)(uint32_t)n) >> 32);",
        "return (int32_t)(((uint64_t)x0 * (uint64_t)(uint32_t)(n - 1)) >> 32);",
        [("test_start_city_uniform_chi2", None)]),
    "heur_power_off_by_one": (
        "for (int32_t b = 0; b < beta; ++b) p = p * (double)d;",
        "for (int32_t b = 0; b <= beta; ++b) p = p * (double)d;",
        [("test_heur_hand_values", None), ("test_heur_exact_rational", {"beta": 2})]),
    "tau_squared_dropped": (
        "return t * t; /* alpha == 2 */", "return t; /* alpha == 2 */",
        [("test_choice_alpha_beta", None)]),
    "nn_tour_ties_highest": (
        "if (best < 0 || dist[(int64_t)cur * n + j] < dist[(int64_t)cur * n + best]) best = j;",
        "if (best < 0 || dist[(int64_t)cur * n + j] <= dist[(int64_t)cur * n + best]) best = j;",
        [("test_nn_tour_ties_lowest_index", None)]),
    "nn_tour_no_closing_edge": (
        "    len += dist[(int64_t)cur * n + 0];\n", "",
        [("test_nn_tour_collinear_closed_form", None)]),
    "s64_row2_carry": (
        "else if (row == 2) out[t] = a[t] + x;", "else if (row == 2) out[t] = a[t] + r1;",
        [("test_s64_integers_exact", None), ("test_s64_total_is_pairwise_tree", None)]),
    "s64_row2_association": (
        "else if (row == 2) out[t] = a[t] + x;", "else if (row == 2) out[t] = (a[t] + r1) + r0;",
        [("test_s64_association_hand_values", None)]),
    "s64_row3_association": (
        "else out[t] = (a[t] + r2) + x;", "else out[t] = a[t] + (r2 + x);",
        [("test_s64_association_hand_values", None)]),
    "s64_row3_carry_order": (
        "else out[t] = (a[t] + r2) + x;", "else out[t] = (a[t] + x) + r2;",
        [("test_s64_association_hand_values", None)]),
    "s64_stage_a_crosses_rows": (
        "float left = (pos >= shift) ? a[t - shift] : 0.0f;",
        "float left = (t >= shift) ? a[t - shift] : 0.0f;",
        [("test_s64_integers_exact", None), ("test_s64_total_is_pairwise_tree", None)]),
    "r64_ge_instead_of_gt": (
        "if (p > target) {", "if (p >= target) {",
        [("test_r64_u_zero_takes_first_positive", None),
         ("test_r64_integer_weights_closed_form", None)]),
    "r64_fallback_lowest": (
        "for (int32_t j = n - 1; j >= 0; --j)", "for (int32_t j = 0; j < n; ++j)",
        [("test_r64_zero_total_takes_last_feasible", None)]),
    "r64_block_offset_index": (
        "float e = (b == 0) ? 0.0f : inc[b - 1];", "float e = inc[b];",
        [("test_r64_integer_weights_closed_form", None),
         ("test_r64_stratified_matches_eq1", {"n": 150})]),
    "r64_total_first_block_only": (
        "float total = inc[nb - 1];", "float total = inc[0];",
        [("test_r64_integer_weights_closed_form", None),
         ("test_r64_stratified_matches_eq1", {"n": 150})]),
    "r64_infeasible_weight_kept": (
        "w[t] = (j < n && feasible[j]) ? row[j] : 0.0f;", "w[t] = (j < n) ? row[j] : 0.0f;",
        [("test_r64_integer_weights_closed_form", None),
         ("test_r64_stratified_matches_eq1", {"n": 150})]),
    "construct_no_closing_edge": (
        "    tour[n] = tour[0];\n    len += dist[(int64_t)cur * n + tour[0]];\n    free(feasible);\n"
        "    return len;\n}\n\nvoid oracle_nn_lists",
        "    tour[n] = tour[0];\n    free(feasible);\n    return len;\n}\n\nvoid oracle_nn_lists",
        [("test_tours_are_permutations", {"n": 64, "m": 10})]),
    "construct_start_not_visited": (
        R64_CONSTRUCT_START, R64_CONSTRUCT_START.replace("    feasible[cur] = 0;\n", ""),
        [("test_tours_are_permutations", {"n": 9, "m": 9}),
         ("test_tours_are_permutations", {"n": 64, "m": 10})]),
    "nn_lists_ties_highest": (
        "if (best < 0 || dist[(int64_t)i * n + j] < dist[(int64_t)i * n + best]) best = j;",
        "if (best < 0 || dist[(int64_t)i * n + j] <= dist[(int64_t)i * n + best]) best = j;",
        [("test_nn_lists_match_lexsort", {"layout": "grid"})]),
    "nn_weight_transposed": (
        "cand_w[r] = choice[(int64_t)cur * n + list[r]];",
        "cand_w[r] = choice[(int64_t)list[r] * n + cur];",
        [("test_nn_full_list_reduces_to_full_construction", {"n": 65})]),
    "nn_fallback_ties_highest": (
        "if (next < 0 || choice[(int64_t)cur * n + j] > choice[(int64_t)cur * n + next])",
        "if (next < 0 || choice[(int64_t)cur * n + j] >= choice[(int64_t)cur * n + next])",
        [("test_nn_fallback_takes_largest_choice_lowest_index", None)]),
    "product_draw_word": (
        "return oracle_uniform(out[j % 4]);", "return oracle_uniform(out[0]);",
        [("test_product_uniform_matches_rocrand", "tpf")]),
    "product_counter_word": (
        "const uint32_t ctr[4] = {step, ant, iter, 1u + (uint32_t)j / 4u};",
        "const uint32_t ctr[4] = {step, ant, iter, (uint32_t)j / 4u};",
        [("test_product_uniform_matches_rocrand", "tpf")]),
    "product_argmin": (
        "if (best < 0 || p > best_p) {", "if (best < 0 || p < best_p) {",
        [("test_product_select_ties_exclusions_rounding", None)]),
    "product_ties_highest": (
        "if (best < 0 || p > best_p) {", "if (best < 0 || p >= best_p) {",
        [("test_product_select_ties_exclusions_rounding", None)]),
    "deposit_amount_in_binary32": (
        "float oracle_deposit_amount(int64_t len) { return (float)(1.0 / (double)len); }",
        "float oracle_deposit_amount(int64_t len) { return 1.0f / (float)len; }",
        [("test_deposit_amount_large_lengths", None),
         ("test_deposit_exact_against_fractions", None), ("test_deposit_invariant_large", None)]),
    "deposit_one_orientation": (
        "            D[(int64_t)j * n + i] += dep;\n", "",
        [("test_deposit_exact_against_fractions", None), ("test_deposit_invariant_large", None),
         ("test_single_ant_full_evaporation", None)]),
    "evaporation_keeps_rho": (
        "float keep = (float)(1.0 - (double)rho);", "float keep = rho;",
        [("test_evaporation_closed_form", None), ("test_single_ant_full_evaporation", None)]),
    "evaporation_after_deposit": (
        "tau[c] = (float)((double)evaporated + D[c]);      /* Eq. 3 */",
        "tau[c] = (float)(((double)tau[c] + D[c]) * (double)keep);",
        [("test_single_ant_full_evaporation", None), ("test_evaporation_closed_form", None),
         ("test_update_single_rounding_against_fractions", {"rho": 0.3})]),
    "deposit_sum_rounded_first": (
        "tau[c] = (float)((double)evaporated + D[c]);      /* Eq. 3 */",
        "tau[c] = evaporated + (float)D[c];",
        [("test_update_single_rounding_against_fractions", {"rho": 0.5}),
         ("test_update_single_rounding_against_fractions", {"rho": 0.3})]),
    "choice_not_refreshed": (
        "    free(D);\n    oracle_choice(n, tau, dist, alpha, beta, choice);\n", "    free(D);\n",
        [("test_choice_refreshed_after_update", None)]),
    "best_ties_latest": (
        "if (lens[k] < *best_len) {", "if (lens[k] <= *best_len) {",
        [("test_best_of_strict_and_earliest", None)]),
    "tau0_inverted": (
        "float tau0 = (float)((double)m / (double)cnn);",
        "float tau0 = (float)((double)cnn / (double)m);",
        [("test_nn_tour_collinear_closed_form", None)]),
}


def _build(tmp_dir, text):
    os.makedirs(tmp_dir, exist_ok=True)
    src = os.path.join(tmp_dir, "aco_oracle.c")
    with open(src, "w") as f:
        f.write(text)
    shutil.copy(HDR, os.path.join(tmp_dir, "aco_oracle.h"))
    lib = os.path.join(tmp_dir, "liboracle.so")
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", lib, src, "-lm"], check=True)
    return lib


def _run_pins(lib_path, pin_list, tmp_path_factory):
    """Runs the pins against the library at lib_path; returns the names of
    those that failed."""
    saved = (oracle.LIB_PATH, oracle._lib)
    oracle.LIB_PATH, oracle._lib = lib_path, None
    failed = []
    try:
        for name, args in pin_list:
            fn = getattr(pins, name)
            try:
                if args == "tpf":
                    fn(oracle, tmp_path_factory)
                else:
                    fn(oracle, **(args or {}))
            except AssertionError:
                failed.append(name)
    finally:
        oracle.LIB_PATH, oracle._lib = saved
    return failed


def _all_pins():
    seen, out = set(), []
    for _, _, pl in MUTANTS.values():
        for name, args in pl:
            key = (name, repr(args))
            if key not in seen:
                seen.add(key)
                out.append((name, args))
    return out


def test_unmodified_copy_passes_every_pin_used(tmp_path_factory):
    text = open(SRC).read()
    lib = _build(str(tmp_path_factory.mktemp("oracle_copy")), text)
    assert _run_pins(lib, _all_pins(), tmp_path_factory) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path_factory):
    old, new, pin_list = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site of {name} not found exactly once"
    lib = _build(str(tmp_path_factory.mktemp(name)), text.replace(old, new))
    failed = _run_pins(lib, pin_list, tmp_path_factory)
    assert failed, f"no pin caught {name}"
