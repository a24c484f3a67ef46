"""GPU: the paper's product-and-argmax selection (Section III-A).

Every selection, tour, length and tau must equal the oracle's bit for bit:
on adversarial rows with the draws given (ties inside a lane and across
lanes, zero and subnormal products, no feasible city), over whole runs with
the Philox draws, and at full size (n = m = 2400, sampled ants).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import tsp_inputs
from gpu_helpers import ORACLE_THREADS, assert_same_f32, compare_run, log
from test_gpu_parity import _adversarial_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _product_rows(n, count, rng):
    rows, feas, _ = _adversarial_rows(n, count, rng)
    u = (rng.integers(0, 2**24, size=(count, n)) / 2**24).astype(np.float32)
    kind = rng.integers(0, 9, size=count)
    for q in range(count):
        if kind[q] == 0:  # many equal products across lanes: weights 1, draws from a tiny set
            rows[q] = 1.0
            u[q] = rng.choice(np.array([0.5, 0.25, 0.75], np.float32), size=n)
        elif kind[q] == 1:  # every product zero
            u[q] = 0.0
        elif kind[q] == 2:  # equal weights and equal draws: every feasible city ties
            rows[q] = 0.375
            u[q] = 0.5
        elif kind[q] == 3:  # the largest draw on the last city
            u[q, n - 1] = 1.0 - 2.0**-24
            rows[q, n - 1] = 1.0
        elif kind[q] == 4:  # products near the binary32 tie boundary
            rows[q] = np.float32(1.0 + 2.0**-23)
            u[q] = rng.choice(np.array([1 - 2.0**-23, 1 - 2.0**-24], np.float32), size=n)
        elif kind[q] == 5:  # the largest choice value draws low; smaller ones tie with it
            rows[q] = 0.25
            u[q] = 0.5
            j = rng.integers(0, n)
            rows[q, j], u[q, j] = 1.0, 0.125
        elif kind[q] == 6:  # the largest choice value draws 0; the winner is far below it
            rows[q] = np.float32(0.01)
            j = rng.integers(0, n)
            rows[q, j], u[q, j] = 1.0, 0.0
        elif kind[q] == 7:  # choice values on and around half and an eighth of the largest
            rows[q] = rng.choice(np.array([0.5, 0.125, np.float32(0.5 - 2.0**-25),
                                           np.float32(0.125 - 2.0**-27)], np.float32), size=n)
            u[q] = rng.choice(np.array([0.25, 0.5, 1 - 2.0**-24], np.float32), size=n)
            j = rng.integers(0, n)
            rows[q, j], u[q, j] = 1.0, 0.0625
    none = rng.random(count) < 0.02
    feas[none] = 0  # no feasible city: -1
    return rows, feas, u


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 9, 63, 64, 65, 511, 512, 513, 1000, 2400, 4095, 4096])
def test_product_select_adversarial(n):
    import torch
    from paper_1101_2678_amd import aco

    rng = np.random.default_rng(7000 + n)
    count = 3000 if n <= 1000 else 800
    rows, feas, u = _product_rows(n, count, rng)
    log(f"  product select n={n} count={count}")
    got = aco.test_product_select(torch.from_numpy(rows).cuda(), torch.from_numpy(feas).cuda(),
                                  torch.from_numpy(u).cuda()).cpu().numpy()
    want = oracle.product_select_batch(rows, feas, u)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} rows differ, first {bad[:5].tolist()}: " \
                          f"got {got[bad[:5]].tolist()} want {want[bad[:5]].tolist()}"


@pytest.mark.parametrize("n,m,layout,alpha,beta,rho,seed", [
    (3, 5, "uniform", 1, 2, 0.5, 1),
    (8, 8, "uniform", 1, 2, 0.5, 2),
    (64, 64, "cluster", 1, 2, 0.5, 3),
    (65, 30, "uniform", 2, 3, 0.3, 4),
    (100, 100, "uniform", 1, 2, 0.5, 5),
    (257, 40, "cluster", 0, 2, 0.9, 6),
    (513, 30, "uniform", 1, 4, 0.5, 7),
    (1000, 40, "uniform", 1, 2, 0.5, 8),
])
def test_product_parity(n, m, layout, alpha, beta, rho, seed):
    _, d = tsp_inputs.instance(n, layout, side=1_000_000, seed=seed)
    compare_run(d, m, alpha, beta, rho, seed, iters=3, rule="product")


def test_product_solve_matches_oracle():
    from paper_1101_2678_amd.aco import Colony

    _, d = tsp_inputs.instance(150, "uniform", side=100_000, seed=31)
    st = oracle.solve(d, 50, 1, 2, 0.5, 31, iters=4, threads=ORACLE_THREADS, rule="product")
    for kind in ("gather", "atomic"):
        c = Colony(d, 50, 1, 2, 0.5, 31, atomic=(kind == "atomic"))
        tour, length = c.solve(4, kind, rule="product")
        assert length == st.best_len and (tour == st.best_tour).all()
        assert_same_f32(c.tau(), st.tau, f"{kind} tau")
        c.close()


@pytest.mark.parametrize("layout", ["uniform", "cluster"])
def test_product_full_size_sampled(layout):
    """n = m = 2400, two iterations: every GPU tour is a permutation with the
    recomputed length, and sampled ants equal the oracle's."""
    from paper_1101_2678_amd.aco import Colony

    n = 2400
    _, d = tsp_inputs.instance(n, layout, side=1_000_000, seed=1)
    c = Colony(d, n, 1, 2, 0.5, 1, atomic=False)
    rng = np.random.default_rng(2401)
    for it in range(2):
        ch = c.choice()
        c.construct_product(it)
        tours, lens = c.tours()
        srt = np.sort(tours[:, :-1], axis=1)
        assert (srt == np.arange(n, dtype=np.uint16)).all()
        t64 = tours.astype(np.int64)
        assert (d[t64[:, :-1], t64[:, 1:]].astype(np.int64).sum(axis=1) == lens).all()
        sample = rng.choice(n, 16, replace=False)
        log(f"  product n2400 {layout} it={it} ants {sample[:4].tolist()}...")
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(ORACLE_THREADS) as ex:
            refs = list(ex.map(lambda k: oracle.construct_ant_product(ch, d, 1, it, int(k)),
                               sample))
        for k, (t, ln) in zip(sample, refs):
            assert (tours[k] == t).all() and lens[k] == ln, f"ant {k} differs"
        c.update("gather")
    c.close()
