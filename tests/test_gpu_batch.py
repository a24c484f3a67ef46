"""GPU: construction tiles, batches and graph replays.

Every instance must compute exactly what it computes alone and what the
oracle computes, whatever tile (cities per lane) the construction kernel
uses, whatever batch it runs in, and whether the batch's launches run
directly or as replays of a captured HIP graph.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import tsp_inputs
from gpu_helpers import ORACLE_THREADS, assert_same_f32, compare_run, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_2678_amd import aco

    yield
    aco.reset_tiles()  # leave the default table for later tests


@pytest.fixture
def tile4():
    from paper_1101_2678_amd import aco

    aco.set_tile(1, 1024, 4)
    yield
    aco.reset_tiles()


@pytest.mark.parametrize("n", [1, 3, 63, 64, 65, 255, 256, 257, 700, 1024])
def test_select_tile4_adversarial(n):
    import torch
    from paper_1101_2678_amd import aco
    from test_gpu_parity import _adversarial_rows

    rng = np.random.default_rng(4000 + n)
    rows, feas, u = _adversarial_rows(n, 2000, rng)
    args = (torch.from_numpy(rows).cuda(), torch.from_numpy(feas).cuda(), torch.from_numpy(u).cuda())
    got4 = aco.test_select(*args, tile=4).cpu().numpy()
    got8 = aco.test_select(*args, tile=8).cpu().numpy()
    want = oracle.r64_select_batch(rows, feas, u)
    assert (got4 == want).all() and (got8 == want).all()


@pytest.mark.parametrize("n,m,alpha,beta,rho", [
    (3, 5, 1, 2, 0.5), (100, 100, 1, 2, 0.5), (257, 40, 2, 3, 0.3), (700, 60, 1, 2, 0.5),
    (1024, 50, 0, 2, 0.9),
])
def test_tile4_parity(tile4, n, m, alpha, beta, rho):
    from paper_1101_2678_amd import aco

    assert aco.get_tile(n) == 4
    _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=n + 3)
    compare_run(d, m, alpha, beta, rho, seed=n, iters=3, kinds=("gather",))


def _batch_case():
    """Uneven instances: n from 3 to 2048, varied m, alpha, beta, rho, seed."""
    spec = [(700, 700, 1, 2, 0.5, 11), (3, 4, 1, 2, 0.5, 12), (64, 64, 1, 2, 0.5, 13),
            (65, 30, 2, 1, 0.3, 14), (1000, 200, 1, 2, 0.5, 15), (17, 90, 0, 0, 0.5, 16),
            (2048, 64, 1, 2, 0.2, 17), (513, 513, 1, 3, 0.9, 18), (250, 250, 1, 2, 1.0, 19),
            (129, 1, 1, 2, 0.5, 20)]
    dists, params = [], []
    for (n, m, a, b, r, s) in spec:
        layout = "cluster" if s % 2 else "uniform"
        _, d = tsp_inputs.instance(n, layout, side=1_000_000, seed=s)
        dists.append(d)
        params.append(dict(m=m, alpha=a, beta=b, rho=r, seed=s))
    return dists, params


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("tiles", ["8", "mixed"])
def test_batch_matches_single(graph, tiles):
    from paper_1101_2678_amd import aco
    from paper_1101_2678_amd.aco import Batch, Colony

    aco.set_tile(1, 4096, 8)
    if tiles == "mixed":
        aco.set_tile(1, 300, 4)
    try:
        dists, params = _batch_case()
        iters = 4
        log(f"  batch graph={graph} tiles={tiles}")
        b = Batch(dists, params)
        b.run(2, graph=graph)
        b.run(2, graph=graph)
        b.sync()
        for q, (d, p) in enumerate(zip(dists, params)):
            c = Colony(d, p["m"], p["alpha"], p["beta"], p["rho"], p["seed"], atomic=False)
            c.solve(iters, "gather")
            ct, cl = c.tours()
            bt, bl = b.tours(q)
            assert (ct == bt).all() and (cl == bl).all(), f"instance {q}: tours differ"
            assert_same_f32(b.tau(q), c.tau(), f"instance {q} tau")
            assert b.best(q)[1] == c.best()[1]
            assert (b.best(q)[0] == c.best()[0]).all()
            assert b.iteration(q) == iters
            c.close()
        b.close()
    finally:
        aco.reset_tiles()


@pytest.mark.parametrize("max_n", [1024, 1025, 2048, 2049, 3072, 3073, 4096])
def test_batch_pass_bounds(max_n):
    """The batched kernel is instantiated for rows of at most 2, 4, 6 or 8
    passes of 512 cities, picked from the batch's largest n: batches whose
    largest instance sits on each side of every bound, with small tile-4
    instances beside it, equal their standalone runs bit for bit."""
    from paper_1101_2678_amd import aco
    from paper_1101_2678_amd.aco import Batch, Colony

    aco.set_tile(1, 200, 4)
    try:
        spec = [(max_n, 6, 31), (150, 40, 32), (513, 9, 33), (7, 5, 34)]
        dists, params = [], []
        for n, m, s in spec:
            _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=s)
            dists.append(d)
            params.append(dict(m=m, alpha=1, beta=2, rho=0.5, seed=s))
        log(f"  batch pass bound max_n={max_n}")
        b = Batch(dists, params)
        b.run(2, graph=False)
        b.sync()
        for q, (d, p) in enumerate(zip(dists, params)):
            c = Colony(d, p["m"], p["alpha"], p["beta"], p["rho"], p["seed"], atomic=False)
            c.solve(2, "gather")
            ct, cl = c.tours()
            bt, bl = b.tours(q)
            assert (ct == bt).all() and (cl == bl).all(), f"instance {q}: tours differ"
            assert_same_f32(b.tau(q), c.tau(), f"instance {q} tau")
            c.close()
        b.close()
    finally:
        aco.reset_tiles()


def test_batch256_full_size():
    """The benchmark's batch in the benchmark's launch configuration: 256
    instances, n = round(exp(U(ln 50, ln 1000))) from seed 4, m = n, uniform
    cities, instance q with seed q + 1, tile 4 up to n = 256 as the tuner
    picks, one captured graph over 2 iterations (81,903 ants per launch, so
    the occupancy cap of long launches is in force).  Every instance's tours,
    lengths and tau equal its standalone run; the four smallest also equal the
    oracle."""
    from paper_1101_2678_amd import aco
    from paper_1101_2678_amd.aco import Batch, Colony

    sizes = tsp_inputs.log_uniform_sizes(256, 50, 1000, seed=4)
    assert int(sizes.sum()) == 81_903
    dists = [tsp_inputs.instance(int(n), "uniform", side=1_000_000, seed=q + 1)[1]
             for q, n in enumerate(sizes)]
    params = [dict(m=int(n), alpha=1, beta=2, rho=0.5, seed=q + 1) for q, n in enumerate(sizes)]
    aco.set_tile(1, 256, 4)
    try:
        log("  batch256 full size, graph, 2 iterations")
        b = Batch(dists, params)
        b.run(2, graph=True)
        b.sync()
        for q, (d, p) in enumerate(zip(dists, params)):
            c = Colony(d, p["m"], 1, 2, 0.5, p["seed"], atomic=False)
            c.solve(2, "gather")
            ct, cl = c.tours()
            bt, bl = b.tours(q)
            assert (ct == bt).all() and (cl == bl).all(), f"instance {q}: tours differ"
            assert_same_f32(b.tau(q), c.tau(), f"instance {q} tau")
            c.close()
        for q in np.argsort(sizes)[:4].tolist():
            st = oracle.solve(dists[q], params[q]["m"], 1, 2, 0.5, params[q]["seed"], 2,
                              threads=ORACLE_THREADS)
            assert_same_f32(b.tau(q), st.tau, f"instance {q} tau vs oracle")
            assert b.best(q)[1] == st.best_len
        b.close()
    finally:
        aco.reset_tiles()


def test_batch_against_oracle():
    """A small batch checked directly against the oracle, instance by instance."""
    from paper_1101_2678_amd.aco import Batch

    dists, params = [], []
    for n, m, s in [(30, 30, 1), (5, 7, 2), (130, 50, 3)]:
        _, d = tsp_inputs.instance(n, "uniform", side=10_000, seed=s)
        dists.append(d)
        params.append(dict(m=m, alpha=1, beta=2, rho=0.5, seed=s))
    b = Batch(dists, params)
    b.run(3, graph=True)
    b.sync()
    for q, (d, p) in enumerate(zip(dists, params)):
        st = oracle.solve(d, p["m"], 1, 2, 0.5, p["seed"], 3, threads=ORACLE_THREADS)
        assert_same_f32(b.tau(q), st.tau, f"instance {q} tau vs oracle")
        assert b.best(q)[1] == st.best_len
    b.close()


def test_graph_replays_with_eager_work_between():
    """Replays of one captured graph, with other launches and host syncs in
    between, advance exactly like eager launches."""
    import torch
    from paper_1101_2678_amd.aco import Batch

    dists, params = _batch_case()
    g = Batch(dists, params)
    e = Batch(dists, params)
    for r in range(4):
        g.run(1, graph=True)
        x = torch.randn(1 << 20, device="cuda")  # unrelated eager work
        torch.cuda.synchronize()
        _ = float(x.sum())
        e.run(1, graph=False)
        g.sync()
        e.sync()
        for q in range(len(dists)):
            assert_same_f32(g.tau(q), e.tau(q), f"replay {r} instance {q}")
            assert g.iteration(q) == e.iteration(q) == r + 1
    g.close()
    e.close()


def test_autotune_sets_table_and_keeps_results():
    """The autotuner times every shape that supports each size, fills the
    shape table with the fastest, and the chosen shapes give the oracle's
    results."""
    from paper_1101_2678_amd import aco

    try:
        tiles, waves, ms = aco.autotune([128, 512, 1000, 2400], reps=2)
        log(f"  autotune tiles={tiles.tolist()} waves={waves.tolist()} ms={ms.tolist()}")
        assert set(tiles.tolist()) <= {4, 8} and set(waves.tolist()) <= {1, 2, 4}
        supported = ms > 0
        # (4, 1) (8, 1) (8, 2) (4, 2) (4, 4) per size
        assert supported.tolist() == [[True, True, False, False, False],
                                      [True, True, False, True, False],
                                      [True, True, True, True, True],
                                      [False, True, False, False, False]]
        for i, n in enumerate((128, 512, 1000, 2400)):
            k = aco.SHAPES.index((int(tiles[i]), int(waves[i])))
            assert ms[i, k] == ms[i][supported[i]].min()
            assert aco.get_tile(n) == tiles[i] and aco.get_waves(n) == waves[i]
        assert aco.get_tile(4096) == 8 and aco.get_waves(4096) == 1
        for n in (300, 1000):
            _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=9)
            compare_run(d, 80, 1, 2, 0.5, 9, 2, kinds=("gather",))
    finally:
        aco.reset_tiles()


def test_batch_configs_same_bits():
    """The batched launch configuration (per-CU workgroup cap, tile per size)
    changes speed only: from a fresh batch, every candidate configuration
    gives the tours, lengths, tau and best tour of the default one, bit for
    bit, over 3 iterations; the autotuner keeps one of the candidates and the
    batch goes on computing exactly what a fresh batch computes."""
    from paper_1101_2678_amd import aco

    dists, params = _batch_case()
    ref = aco.Batch(dists, params)
    ref.run(3, graph=False)
    ref.sync()
    want = [(ref.tours(q), ref.tau(q), ref.best(q)) for q in range(len(dists))]
    ref.close()
    cands = [(0, -1), (3, -1), (8, 0), (16, 1024), (24, 256), (64, 0)]
    for cfg in cands:
        log(f"  batch config wg_per_cu={cfg[0]} tile4_max_n={cfg[1]}")
        b = aco.Batch(dists, params)
        b.set_config(*cfg)
        assert b.config == {"wg_per_cu": cfg[0], "tile4_max_n": cfg[1]}
        b.run(3, graph=True)
        b.sync()
        for q in range(len(dists)):
            (wt, wl), wtau, (wbt, wbl) = want[q]
            gt, gl = b.tours(q)
            assert (gt == wt).all() and (gl == wl).all(), f"config {cfg}: instance {q} tours"
            assert_same_f32(b.tau(q), wtau, f"config {cfg}: instance {q} tau")
            bt, bl = b.best(q)
            assert bl == wbl and (bt == wbt).all()
        b.close()
    # the autotuner: 6 candidates x (1 + 1) iterations, then 2 more iterations,
    # against a fresh batch run for the same 14 iterations
    b = aco.Batch(dists, params)
    best, ms = b.autotune(cands, iters=1)
    assert 0 <= best < len(cands) and (ms > 0).all()
    assert b.config == {"wg_per_cu": cands[best][0], "tile4_max_n": cands[best][1]}
    b.run(2, graph=True)
    b.sync()
    fresh = aco.Batch(dists, params)
    fresh.run(14, graph=False)
    fresh.sync()
    for q in range(len(dists)):
        assert b.iteration(q) == 14
        assert_same_f32(b.tau(q), fresh.tau(q), f"autotuned batch: instance {q} tau")
        assert b.best(q)[1] == fresh.best(q)[1]
    with pytest.raises(aco.AcoError) as e:
        b.set_config(65, -1)
    assert e.value.status == aco.ACO_ERR_INVALID
    with pytest.raises(aco.AcoError) as e:
        b.set_config(0, 1025)
    assert e.value.status == aco.ACO_ERR_INVALID
    b.close()
    fresh.close()
