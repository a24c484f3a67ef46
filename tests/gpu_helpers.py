"""Shared pieces of the GPU parity tests: run the HIP library and the oracle
on the same seeded instance and compare what both produce."""
from __future__ import annotations

import os
import sys

import numpy as np

import oracle
import tsp_inputs

# host threads the oracle may use to construct ants in parallel (each ant is
# still one serial oracle call, so results do not depend on it)
ORACLE_THREADS = min(16, os.cpu_count() or 1)


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def tour_length(d: np.ndarray, tour: np.ndarray) -> int:
    t = np.asarray(tour, np.int64)
    return int(d[t[:-1], t[1:]].astype(np.int64).sum())


def bits(a) -> np.ndarray:
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def assert_same_f32(got, want, what: str):
    g, w = bits(got), bits(want)
    bad = np.argwhere(g != w)
    assert bad.size == 0, (f"{what}: {len(bad)} cells differ, first {bad[:3].tolist()} "
                           f"got {np.asarray(got)[tuple(bad[0])]!r} want "
                           f"{np.asarray(want)[tuple(bad[0])]!r}")


def compare_run(dist, m, alpha, beta, rho, seed, iters, kinds=("gather", "atomic"),
                check_choice=True, nn=None, rule="r64"):
    """Full parity: every iteration's tours, lengths, tau (and choice)
    bit-exact.  nn: construct over candidate lists of that length (the lists
    themselves are compared first); rule "product": the product-and-argmax
    selection."""
    from paper_1101_2678_amd.aco import Colony

    n = dist.shape[0]
    log(f"  parity n={n} m={m} alpha={alpha} beta={beta} rho={rho} seed={seed} iters={iters} "
        f"nn={nn} rule={rule}")
    ref = oracle.init(dist, m, alpha, beta, rho, seed)
    cols = {k: Colony(dist, m, alpha, beta, rho, seed, atomic=(k != "gather")) for k in kinds}
    nnl = None
    if nn is not None:
        nnl = oracle.nn_lists(dist, nn)
        for k, col in cols.items():
            col.attach_nn(nn)
            got = col.nn_lists()
            bad = np.nonzero((got != nnl).any(axis=1))[0]
            assert bad.size == 0, f"{k}: candidate lists of rows {bad[:5].tolist()} differ"
    for k, col in cols.items():
        assert_same_f32(col.tau(), ref.tau, f"{k} tau0")
        if check_choice:
            assert_same_f32(col.choice(), ref.choice, f"{k} initial choice")
    for it in range(iters):
        if rule == "product":
            tours, lens = oracle.construct_product(ref.choice, dist, m, seed, it, ORACLE_THREADS)
        elif nnl is None:
            tours, lens = oracle.construct(ref.choice, dist, m, seed, it, ORACLE_THREADS)
        else:
            tours, lens = oracle.construct_nn(ref.choice, dist, nnl, m, seed, it,
                                              ORACLE_THREADS)
        import ctypes

        best = ctypes.c_int64(ref.best_len)
        who = oracle.lib().oracle_best_of(m, lens, ctypes.byref(best))
        if who >= 0:
            ref.best_len, ref.best_tour = int(best.value), tours[who].copy()
        ref.tau, ref.choice = oracle.update(ref.tau, tours, lens, dist, rho, alpha, beta)
        ref.it += 1
        for k, col in cols.items():
            if rule == "product":
                col.construct_product(it)
            elif nnl is None:
                col.construct(it)
            else:
                col.construct_nn(it)
            gt, gl = col.tours()
            bad = np.nonzero((gt != tours).any(axis=1))[0]
            assert bad.size == 0, f"{k} it={it}: tours of ants {bad[:5].tolist()} differ"
            assert (gl == lens).all(), f"{k} it={it}: lengths differ"
            col.update(k)
            assert_same_f32(col.tau(), ref.tau, f"{k} it={it} tau")
            if check_choice:
                assert_same_f32(col.choice(), ref.choice, f"{k} it={it} choice")
    for k, col in cols.items():
        bt, bl = col.best()
        assert bl == ref.best_len, f"{k}: best length {bl} != {ref.best_len}"
        assert (bt == ref.best_tour).all(), f"{k}: best tour differs"
        assert col.iteration == iters
        col.close()
    return ref
