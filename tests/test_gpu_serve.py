"""GPU: continuous batching.  Every request served in a changing mix must
give exactly the result it gives alone; admission follows slots, table
limits and pool memory."""
from __future__ import annotations

import time

import numpy as np
import pytest

import tsp_inputs
from gpu_helpers import assert_same_f32, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _requests(count, seed, n_lo=20, n_hi=400, rate=3000.0):
    from paper_1101_2678_amd.serve import make_requests

    reqs = make_requests(count, rate, n_lo=n_lo, n_hi=n_hi, iters=8, seed=seed)
    for r in reqs:  # uneven iteration counts so that requests leave at different ticks
        r.iters = 4 + (r.rid * 5) % 9
    return reqs


def test_served_results_equal_alone():
    from paper_1101_2678_amd.aco import Colony
    from paper_1101_2678_amd.serve import Server, run_open_loop

    reqs = _requests(12, seed=21)
    srv = Server(pool_bytes=256 << 20, max_slots=4)
    summary = run_open_loop(srv, reqs, keep_tau=True)
    log(f"  served: {summary}")
    assert summary["peak_running"] >= 2  # the mix really overlapped
    for r in reqs:
        c = Colony(r.dist, r.m, r.alpha, r.beta, r.rho, r.seed, atomic=False)
        tour, length = c.solve(r.iters, "gather")
        assert length == r.best_len, f"request {r.rid}: {r.best_len} != {length}"
        assert (tour == r.best_tour).all()
        assert_same_f32(r.extra["tau"], c.tau(), f"request {r.rid} tau")
        c.close()
    assert srv.stats()["running"] == 0 and srv.stats()["finished"] == 0
    srv.close()


def test_served_results_match_oracle():
    """Requests served in a mix against the oracle directly (not only against
    the library's own standalone path): small instances with uneven iteration
    counts, both layouts, and two above 1000 cities, all running at once; each
    best tour, best length and final tau bit-exact against oracle.solve with
    the request's parameters and seed (Section II, Eqs. 1-4)."""
    import oracle
    from gpu_helpers import ORACLE_THREADS
    from paper_1101_2678_amd.serve import Request, Server, run_open_loop

    specs = [(17, "uniform", 6), (64, "cluster", 3), (150, "uniform", 9), (333, "cluster", 5),
             (700, "uniform", 4), (1100, "cluster", 3), (1500, "uniform", 2)]
    reqs = []
    for q, (n, layout, iters) in enumerate(specs):
        _, d = tsp_inputs.instance(n, layout, side=1_000_000, seed=300 + q)
        reqs.append(Request(rid=q, arrival=0.0, dist=d, m=n, iters=iters, seed=77 + 13 * q,
                            layout=layout))
    srv = Server(pool_bytes=1 << 30, max_slots=8)
    summary = run_open_loop(srv, reqs, keep_tau=True)
    srv.close()
    log(f"  served vs oracle: {summary}")
    assert summary["peak_running"] >= 4
    for r in reqs:
        st = oracle.solve(r.dist, r.m, r.alpha, r.beta, r.rho, r.seed, r.iters,
                          threads=ORACLE_THREADS)
        assert r.best_len == st.best_len, f"request {r.rid} (n={r.n}): {r.best_len} != {st.best_len}"
        assert (r.best_tour == st.best_tour).all(), f"request {r.rid}: best tour differs"
        assert_same_f32(r.extra["tau"], st.tau, f"request {r.rid} (n={r.n}) tau")


def test_served_trace_at_benchmark_sizes():
    """The first 30 requests of the benchmark's trace (Poisson 200/s, n
    log-uniform in [100, 3000], both layouts, 50 iterations each, per-request
    seeds) through the default server (size classes, 32 slots, a pool of half
    the free memory): every best tour and length equals the request run
    alone with a context of its own."""
    import copy

    from paper_1101_2678_amd.serve import Server, make_requests, run_open_loop, run_plain

    reqs = make_requests(30, 200.0, n_lo=100, n_hi=3000, iters=50, seed=5)
    alone = copy.deepcopy(reqs)
    srv = Server(max_slots=32)
    summary = run_open_loop(srv, reqs)
    srv.close()
    log(f"  served at benchmark sizes: {summary}")
    assert summary["peak_running"] >= 8  # overlapping requests in several classes
    run_plain(alone)
    for a, b in zip(reqs, alone):
        assert a.best_len == b.best_len, f"request {a.rid} (n={a.n}): {a.best_len} != {b.best_len}"
        assert (a.best_tour == b.best_tour).all(), f"request {a.rid}: tours differ"


def test_admission_waits_for_memory():
    """A pool that fits one request at a time: the second is refused until the
    first is released, and both still give their standalone results."""
    from paper_1101_2678_amd.aco import Colony, workspace_bytes
    from paper_1101_2678_amd.serve import Request, Server

    _, d1 = tsp_inputs.instance(300, "uniform", side=1_000_000, seed=1)
    _, d2 = tsp_inputs.instance(280, "cluster", side=1_000_000, seed=2)
    r1 = Request(rid=1, arrival=0.0, dist=d1, m=300, iters=5, seed=3)
    r2 = Request(rid=2, arrival=0.0, dist=d2, m=280, iters=5, seed=4)
    from paper_1101_2678_amd.aco import lib

    classes = (512, 1024, 2048, 4096)
    head = lib.aco_server_table_bytes(4, 4096, 4096, len(classes))
    pool = head + workspace_bytes(300, 300, atomic=False) + 4096
    srv = Server(pool_bytes=pool, max_slots=4, max_ants=4096, max_rows=4096,
                 class_max_n=classes)
    s1 = srv.submit(r1)
    assert s1 is not None
    assert srv.submit(r2) is None  # no room
    while True:
        srv.step()
        done = srv.collect()
        if done:
            break
        time.sleep(1e-4)
    assert done == [(s1, 1)]
    r1.best_tour, r1.best_len = srv.result(s1, 300)
    assert srv.submit(r2) is None  # still held until released
    srv.release(s1)
    s2 = srv.submit(r2)
    assert s2 is not None
    while not srv.collect():
        srv.step()
        time.sleep(1e-4)
    r2.best_tour, r2.best_len = srv.result(s2, 280)
    srv.release(s2)
    for r in (r1, r2):
        c = Colony(r.dist, r.m, 1, 2, 0.5, r.seed, atomic=False)
        assert c.solve(r.iters)[1] == r.best_len
        c.close()
    srv.close()


def test_admission_respects_table_limits():
    from paper_1101_2678_amd.serve import Request, Server

    _, d = tsp_inputs.instance(100, "uniform", side=10_000, seed=5)
    srv = Server(pool_bytes=64 << 20, max_slots=8, max_ants=150, max_rows=1000)
    a = srv.submit(Request(rid=1, arrival=0, dist=d, m=100, iters=2, seed=1))
    b = srv.submit(Request(rid=2, arrival=0, dist=d, m=100, iters=2, seed=2))
    assert a is not None and b is None  # 200 ants > 150 in one size class
    _, d2 = tsp_inputs.instance(600, "uniform", side=10_000, seed=6)
    c = srv.submit(Request(rid=3, arrival=0, dist=d2, m=100, iters=2, seed=3))
    assert c is not None  # another size class has its own capacity
    srv.close()


def test_small_requests_not_paced_by_large():
    """A small request submitted beside a large one finishes first: each size
    class ticks on its own."""
    from paper_1101_2678_amd.serve import Request, Server

    _, big = tsp_inputs.instance(2400, "uniform", side=1_000_000, seed=7)
    _, small = tsp_inputs.instance(100, "uniform", side=1_000_000, seed=8)
    srv = Server(pool_bytes=1 << 30, max_slots=4)
    sb = srv.submit(Request(rid=1, arrival=0, dist=big, m=2400, iters=6, seed=1))
    ss = srv.submit(Request(rid=2, arrival=0, dist=small, m=100, iters=6, seed=2))
    order = []
    while len(order) < 2:
        srv.step()
        order += [rid for _, rid in srv.collect()]
        time.sleep(1e-4)
    assert order == [2, 1], order
    srv.close()
