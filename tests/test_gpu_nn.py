"""GPU: construction over nearest-neighbour candidate lists.

The lists, every tour and length, and tau after each update must equal the
oracle's bit for bit, on instances whose lists have ties (grids), that
need the fallback often (nn = 1), at the list lengths of the paper (30) and
the kernel's limit (64), and at full size (n = m = 2400, sampled ants).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import tsp_inputs
from gpu_helpers import ORACLE_THREADS, compare_run, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _grid(rows, cols, step=10):
    xy = np.array([[step * c, step * r] for r in range(rows) for c in range(cols)], np.int64)
    return tsp_inputs.euc2d(xy)


@pytest.mark.parametrize("n,layout,nn", [
    (3, "uniform", 1), (3, "uniform", 2), (40, "grid", 7), (65, "uniform", 64),
    (300, "cluster", 30), (1000, "uniform", 30), (4096, "uniform", 64), (2048, "grid", 30),
])
def test_nn_lists(n, layout, nn):
    from paper_1101_2678_amd.aco import Colony

    d = _grid(32, n // 32) if layout == "grid" and n % 32 == 0 else (
        _grid(5, 8) if layout == "grid" else
        tsp_inputs.instance(n, layout, side=1_000_000, seed=n)[1])
    log(f"  nn lists n={d.shape[0]} layout={layout} nn={nn}")
    c = Colony(d, 4, 1, 2, 0.5, 1, atomic=False)
    c.attach_nn(nn)
    got = c.nn_lists()
    want = oracle.nn_lists(d, nn)
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert bad.size == 0, f"rows {bad[:5].tolist()} differ"
    c.close()


@pytest.mark.parametrize("n,m,nn,layout,alpha,beta,rho,seed", [
    (3, 5, 1, "uniform", 1, 2, 0.5, 1),
    (3, 2, 2, "uniform", 1, 2, 0.5, 2),
    (64, 64, 30, "uniform", 1, 2, 0.5, 3),
    (65, 20, 64, "cluster", 1, 2, 0.5, 4),
    (100, 100, 30, "uniform", 1, 2, 0.5, 5),
    (130, 40, 1, "cluster", 1, 2, 0.5, 6),   # fallback at most steps
    (257, 50, 15, "uniform", 2, 3, 0.3, 7),
    (40, 30, 7, "grid", 1, 2, 0.5, 8),       # ties in lists and fallback
    (700, 64, 30, "cluster", 0, 2, 0.9, 9),
    (1000, 100, 40, "uniform", 1, 2, 0.5, 10),
])
def test_nn_parity(n, m, nn, layout, alpha, beta, rho, seed):
    d = _grid(5, 8) if layout == "grid" else tsp_inputs.instance(
        n, layout, side=1_000_000, seed=seed)[1]
    compare_run(d, m, alpha, beta, rho, seed, iters=3, nn=nn)


def test_nn_solve_matches_oracle():
    from paper_1101_2678_amd.aco import Colony

    _, d = tsp_inputs.instance(150, "uniform", side=100_000, seed=21)
    st = oracle.solve(d, 60, 1, 2, 0.5, 21, iters=5, threads=ORACLE_THREADS, nn=20)
    for kind in ("gather", "atomic"):
        c = Colony(d, 60, 1, 2, 0.5, 21, atomic=(kind == "atomic"))
        c.attach_nn(20)
        tour, length = c.solve(5, kind, rule="nn")
        assert length == st.best_len and (tour == st.best_tour).all()
        assert (c.tau().view(np.uint32) == st.tau.view(np.uint32)).all()
        c.close()


def test_nn_then_full_construction_share_state():
    """Switching rules between iterations: the state after nn, full, nn
    iterations equals the oracle's run of the same sequence."""
    from paper_1101_2678_amd.aco import Colony

    _, d = tsp_inputs.instance(200, "cluster", side=100_000, seed=22)
    nnl = oracle.nn_lists(d, 30)
    st = oracle.init(d, 50, 1, 2, 0.5, 22)
    c = Colony(d, 50, 1, 2, 0.5, 22, atomic=False)
    c.attach_nn(30)
    for it, rule in enumerate(["nn", "r64", "nn"]):
        oracle.iterate(st, d, ORACLE_THREADS, nnl=nnl if rule == "nn" else None)
        (c.construct_nn if rule == "nn" else c.construct)(it)
        c.update("gather")
        assert (c.tau().view(np.uint32) == st.tau.view(np.uint32)).all(), (it, rule)
    assert c.best()[1] == st.best_len
    c.close()


@pytest.mark.parametrize("layout", ["uniform", "cluster"])
def test_nn_full_size_sampled(layout):
    """n = m = 2400, nn = 30, two iterations: every GPU tour is a
    permutation with the recomputed length, and sampled ants equal the
    oracle's, constructed one by one from the same choice matrix."""
    from paper_1101_2678_amd.aco import Colony

    n = 2400
    _, d = tsp_inputs.instance(n, layout, side=1_000_000, seed=1)
    c = Colony(d, n, 1, 2, 0.5, 1, atomic=False)
    c.attach_nn(30)
    nnl = oracle.nn_lists(d, 30)
    assert (c.nn_lists() == nnl).all()
    rng = np.random.default_rng(2400)
    for it in range(2):
        ch = c.choice()
        c.construct_nn(it)
        tours, lens = c.tours()
        srt = np.sort(tours[:, :-1], axis=1)
        assert (srt == np.arange(n, dtype=np.uint16)).all()
        assert (tours[:, 0] == tours[:, -1]).all()
        t64 = tours.astype(np.int64)
        assert (d[t64[:, :-1], t64[:, 1:]].astype(np.int64).sum(axis=1) == lens).all()
        sample = rng.choice(n, 24, replace=False)
        log(f"  n2400 {layout} it={it} ants {sample[:4].tolist()}...")
        for k in sample:
            t, ln = oracle.construct_ant_nn(ch, d, nnl, 1, it, int(k))
            assert (tours[k] == t).all() and lens[k] == ln, f"ant {k} differs"
        c.update("gather")
    assert (c.nn_lists() == nnl).all()  # the lists are never written after attach
    c.close()


def test_nn_entry_points_validate():
    """Misuse of the candidate-list entry points is refused with the
    documented status and leaves the context usable."""
    import ctypes

    import torch
    from paper_1101_2678_amd import aco
    from paper_1101_2678_amd.aco import (ACO_ERR_INVALID, ACO_ERR_NOMEM, ACO_ERR_STATE, AcoError,
                                         Colony)

    _, d = tsp_inputs.instance(40, "uniform", side=10_000, seed=44)
    c = Colony(d, 10, 1, 2, 0.5, 44, atomic=False)
    with pytest.raises(AcoError) as e:
        c.construct_nn(0)                       # no lists attached yet
    assert e.value.status == ACO_ERR_STATE
    with pytest.raises(AcoError) as e:
        c.solve(1, "gather", rule="nn")
    assert e.value.status == ACO_ERR_STATE
    for bad in (0, 40, 65):                     # nn must be in [1, min(64, n - 1)]
        with pytest.raises(AcoError) as e:
            c.attach_nn(bad)
        assert e.value.status == ACO_ERR_INVALID
    need = aco.lib.aco_nn_workspace_bytes(40, 30)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    base = ws.data_ptr() + (-ws.data_ptr()) % 256
    assert aco.lib.aco_nn_attach(c._ctx, 30, ctypes.c_void_p(base), need - 1) == ACO_ERR_NOMEM
    assert aco.lib.aco_nn_attach(c._ctx, 30, ctypes.c_void_p(base + 16), need) == ACO_ERR_NOMEM
    c.attach_nn(39)                             # the largest list for n = 40 works
    c.construct_nn(0)
    c.update("gather")
    t, ln = c.tours()
    assert (np.sort(t[:, :-1], axis=1) == np.arange(40)).all()
    c.close()
