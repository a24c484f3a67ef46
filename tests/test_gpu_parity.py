"""GPU parity: the HIP library against the oracle, element by element.

Tours and integer lengths must be identical; tau and choice must be identical
bit for bit for both update variants (the binary64 deposit sums are exact, so
the summation order of the atomics cannot show).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import tsp_inputs
from gpu_helpers import ORACLE_THREADS, assert_same_f32, compare_run, log, tour_length

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


# ------------------------------------------------------------------ R64 roulette
def _adversarial_rows(n, count, rng):
    """Rows with magnitudes from 2^-100 to 1, runs of zeros, sparse and dense
    feasibility, one feasible city, all-zero weights, subnormal weights."""
    rows = (rng.random((count, n)) * np.exp2(rng.integers(-100, 1, size=(count, n)))).astype(
        np.float32)
    kind = rng.integers(0, 8, size=count)
    feas = (rng.random((count, n)) < rng.random((count, 1))).astype(np.uint8)
    for q in range(count):
        if kind[q] == 0:  # runs of zeros
            a = rng.integers(0, n)
            rows[q, a:a + rng.integers(1, 200)] = 0
        elif kind[q] == 1:  # one feasible city
            feas[q] = 0
            feas[q, rng.integers(0, n)] = 1
        elif kind[q] == 2:  # all weights zero
            rows[q] = 0
        elif kind[q] == 3:  # subnormal weights
            rows[q] = (rng.random(n) * 2.0**-130).astype(np.float32)
        elif kind[q] == 4:  # uniform magnitudes (typical choice rows)
            rows[q] = rng.random(n).astype(np.float32)
        elif kind[q] == 5:  # all feasible
            feas[q] = 1
        elif kind[q] == 6:  # feasible only in the last partial block
            feas[q] = 0
            feas[q, (n - 1) // 64 * 64:] = 1
    feas[feas.sum(axis=1) == 0, n - 1] = 1
    u = (rng.integers(0, 2**24, size=count) / 2**24).astype(np.float32)
    u[::7] = 0.0
    u[3::7] = 1.0 - 2.0**-24
    return rows, feas, u


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 100, 511, 512, 513, 1000, 2400, 4095, 4096])
def test_select_adversarial(n):
    import torch
    from paper_1101_2678_amd import aco

    rng = np.random.default_rng(1000 + n)
    count = 4000 if n <= 1000 else 1000
    rows, feas, u = _adversarial_rows(n, count, rng)
    log(f"  select n={n} count={count}")
    got = aco.test_select(torch.from_numpy(rows).cuda(), torch.from_numpy(feas).cuda(),
                          torch.from_numpy(u).cuda()).cpu().numpy()
    torch.cuda.synchronize()
    want = oracle.r64_select_batch(rows, feas, u)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} rows differ, first {bad[:5].tolist()}"


def test_select_non_monotone_prefix():
    """Rows where an FP32 tree prefix inside a block exceeds later prefixes:
    the GPU must return the same first feasible crossing as the definition."""
    import torch
    from paper_1101_2678_amd import aco

    rng = np.random.default_rng(77)
    rows, us = [], []
    while len(rows) < 300:
        w = rng.random(64).astype(np.float32)
        w[63] = 0
        s = oracle.s64(w)
        if (s[:63] > s[63]).any():
            rows.append(np.concatenate([rng.random(64).astype(np.float32), w]))
            us.append(np.float32(1.0 - 2.0**-24))
    rows = np.array(rows)
    feas = np.ones_like(rows, dtype=np.uint8)
    u = np.array(us, np.float32)
    got = aco.test_select(torch.from_numpy(rows).cuda(), torch.from_numpy(feas).cuda(),
                          torch.from_numpy(u).cuda()).cpu().numpy()
    assert (got == oracle.r64_select_batch(rows, feas, u)).all()


# ------------------------------------------------------------------ full solves
def test_parity_config_n100():
    """n = m = 100, uniform in [0, 10^4]^2, alpha 1, beta 2, rho 0.5, seed 1,
    10 iterations: every tour, length, tau and choice bit-exact."""
    _, d = tsp_inputs.instance(100, "uniform", side=10_000, seed=1)
    compare_run(d, 100, 1, 2, 0.5, 1, 10, kinds=("gather", "atomic", "atomic_direct"))


@pytest.mark.parametrize("n,m,alpha,beta,rho", [
    (3, 4, 1, 2, 0.5), (5, 1, 1, 2, 1.0), (17, 33, 2, 4, 0.3), (63, 63, 1, 2, 0.5),
    (64, 10, 0, 0, 0.5), (65, 65, 1, 0, 0.9), (127, 50, 0, 1, 0.5), (129, 129, 2, 1, 0.2),
    (511, 40, 1, 2, 0.5), (512, 31, 1, 3, 0.5), (513, 64, 1, 2, 0.5), (600, 100, 1, 2, 0.1),
])
def test_parity_ragged(n, m, alpha, beta, rho):
    _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=n)
    compare_run(d, m, alpha, beta, rho, seed=n + 7, iters=3,
                kinds=("gather", "atomic", "atomic_direct"))


@pytest.mark.parametrize("n", [1025, 1536, 1537, 2048])
def test_parity_three_and_four_passes(n):
    """Rows of three and four 512-city passes, where construction skips the
    loads of city quads that are all visited: every tour, length, tau and
    choice bit-exact over 3 iterations, both update variants."""
    _, d = tsp_inputs.instance(n, "cluster", side=1_000_000, seed=n)
    compare_run(d, 40, 1, 2, 0.5, seed=n + 3, iters=3)


@pytest.mark.parametrize("n", [2049, 2113, 3000])
def test_parity_five_and_six_passes(n):
    """Rows of five and six 512-city passes around the first ragged sizes
    past 2048 (ld = 2112, 2112, 3008) and with more LDS accumulators per
    gather workgroup than at n = 2400: every tour, length, tau and choice
    bit-exact over 3 iterations, gather and atomic."""
    _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=n)
    compare_run(d, 40, 1, 2, 0.5, seed=n + 5, iters=3)


@pytest.mark.parametrize("m", [2047, 2048, 3001])
def test_parity_many_ants(m):
    """Colonies on each side of the ant count from which both LDS-combining
    updates sum the deposits to the shared neighbours in registers, over
    enough iterations for most ants to share them: every tour, length, tau
    and choice bit-exact, gather and atomic."""
    _, d = tsp_inputs.instance(60, "cluster", side=100_000, seed=m)
    compare_run(d, m, 1, 2, 0.5, seed=m + 11, iters=8)


@pytest.mark.parametrize("layout", ["uniform", "cluster"])
def test_parity_n1000_full(layout):
    """The n = m = 1000 workload in full (both layouts, instance seed 1,
    alpha 1, beta 2, rho 0.5, Philox seed 1, 20 iterations): every tour,
    length, tau and choice of every iteration bit-exact against the oracle,
    with the gather and the atomic update, in the launch configuration the
    benchmark times."""
    _, d = tsp_inputs.instance(1000, layout, side=1_000_000, seed=1)
    compare_run(d, 1000, 1, 2, 0.5, 1, 20, kinds=("gather", "atomic", "atomic_direct"))


def test_subnormal_choice_values():
    """alpha 2, beta 4 on a large square drive tau^2 * eta^4 into the binary32
    subnormal range; nothing may be flushed to zero."""
    _, d = tsp_inputs.instance(200, "uniform", side=3_000_000, seed=5)
    ref = compare_run(d, 50, 2, 4, 0.5, 3, 2)
    ch = ref.choice[~np.eye(200, dtype=bool)]
    assert (ch[ch > 0] < 2.0**-126).any(), "test does not reach subnormal values"


# ------------------------------------------------------------------ full size, bench launch
def test_parity_n2400_full():
    """The benchmark workload in full (n = m = 2400 uniform in [0, 10^6]^2,
    alpha 1, beta 2, rho 0.5, Philox seed 1, 10 iterations) in the launch
    configuration the benchmark times: every tour, length, tau and choice of
    every iteration bit-exact against the oracle, with the gather and the
    atomic update; then the invariants no oracle is needed for (permutations,
    symmetric tau, cells no tour touched only evaporate)."""
    n = m = 2400
    _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=1)
    ref = compare_run(d, m, 1, 2, 0.5, 1, 10)
    assert (ref.tau.view(np.uint32) == ref.tau.T.view(np.uint32)).all()


def test_n2400_invariants_after_convergence():
    """Iterations 10..12 of the benchmark workload (past the point where most
    ants share the best tour's edges): every tour a permutation with its exact
    length, tau symmetric bit for bit, gather and atomic identical, and cells
    no tour touched exactly tau * 0.5 (Eq. 2)."""
    from paper_1101_2678_amd.aco import Colony

    n = m = 2400
    _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=1)
    g = Colony(d, m, 1, 2, 0.5, 1, atomic=True)
    a = Colony(d, m, 1, 2, 0.5, 1, atomic=True)
    x = Colony(d, m, 1, 2, 0.5, 1, atomic=True)
    for it in range(10):
        g.construct(it)
        g.update("gather")
        a.construct(it)
        a.update("atomic")
        x.construct(it)
        x.update("atomic_direct")
    for it in range(10, 13):
        log(f"  n=2400 iteration {it}")
        tau_before = g.tau()
        g.construct(it)
        a.construct(it)
        gt, gl = g.tours()
        at, al = a.tours()
        assert (gt == at).all() and (gl == al).all()
        assert (np.sort(gt[:, :-1], axis=1) == np.arange(n)).all(), "not a permutation"
        assert (gt[:, 0] == gt[:, -1]).all()
        assert all(tour_length(d, gt[k]) == gl[k] for k in range(m))
        x.construct(it)
        g.update("gather")
        a.update("atomic")
        x.update("atomic_direct")
        tg, ta = g.tau(), a.tau()
        assert_same_f32(tg, ta, f"it={it} gather vs atomic tau")
        assert_same_f32(x.tau(), ta, f"it={it} atomic_direct vs atomic tau")
        assert (tg.view(np.uint32) == tg.T.view(np.uint32)).all()
        untouched = np.ones((n, n), bool)
        idx = gt[:, :-1].astype(np.int64), gt[:, 1:].astype(np.int64)
        untouched[idx[0].ravel(), idx[1].ravel()] = False
        untouched[idx[1].ravel(), idx[0].ravel()] = False
        assert (tg[untouched] == tau_before[untouched] * np.float32(0.5)).all()
    g.close()
    a.close()
    x.close()


def test_restore_resumes_bit_exact_and_validates():
    """Checkpoint and resume: tau, best tour and iteration counter copied out
    after 3 iterations and restored into a fresh context give the same state
    after 2 more iterations as 5 uninterrupted ones (every draw is keyed by
    (seed, iter, ant, step)).  Invalid tau is refused before any device work."""
    from paper_1101_2678_amd.aco import ACO_ERR_INVALID, AcoError, Colony

    _, d = tsp_inputs.instance(300, "cluster", side=100_000, seed=41)
    full = Colony(d, 60, 1, 2, 0.5, 41, atomic=False)
    full.solve(5, "gather")
    part = Colony(d, 60, 1, 2, 0.5, 41, atomic=False)
    part.solve(3, "gather")
    tau, (bt, bl), it = part.tau(), part.best(), part.iteration
    assert it == 3
    resumed = Colony(d, 60, 1, 2, 0.5, 41, atomic=False)
    resumed.restore(tau, it, bl, bt)
    assert resumed.iteration == 3
    assert_same_f32(resumed.choice(), part.choice(), "choice after restore")
    resumed.solve(2, "gather")
    assert_same_f32(resumed.tau(), full.tau(), "tau after resume")
    assert resumed.best()[1] == full.best()[1]
    assert (resumed.best()[0] == full.best()[0]).all()
    for bad in (-1.0, np.nan, np.inf, 2e18):
        t = tau.copy()
        t[5, 7] = bad
        with pytest.raises(AcoError) as e:
            resumed.restore(t, 0)
        assert e.value.status == ACO_ERR_INVALID
    assert_same_f32(resumed.tau(), full.tau(), "tau untouched by refused restores")
    for c in (full, part, resumed):
        c.close()


def test_call_order():
    """An update needs a construction before it: one without, or a second
    one after the same construction, is refused with ACO_ERR_STATE and
    leaves the colony as it was; the sequence then goes on as normal and
    matches the oracle."""
    from paper_1101_2678_amd.aco import ACO_ERR_STATE, AcoError, Colony

    _, d = tsp_inputs.instance(90, "uniform", side=10_000, seed=57)
    c = Colony(d, 20, 1, 2, 0.5, 57, atomic=True)
    tau0 = c.tau()
    for kind in ("gather", "atomic"):
        with pytest.raises(AcoError) as e:
            c.update(kind)
        assert e.value.status == ACO_ERR_STATE
    assert_same_f32(c.tau(), tau0, "tau after refused updates")
    c.construct(0)
    c.update("atomic")
    with pytest.raises(AcoError) as e:
        c.update("gather")
    assert e.value.status == ACO_ERR_STATE
    c.construct(1)
    c.update("gather")
    st = oracle.solve(d, 20, 1, 2, 0.5, 57, 2, threads=ORACLE_THREADS)
    assert_same_f32(c.tau(), st.tau, "tau after two iterations vs oracle")
    assert c.iteration == 2
    c.close()


@pytest.mark.parametrize("rule", ["r64", "nn", "product"])
def test_max_cities_sampled(rule):
    """n = 4096, the largest instance the library accepts (8 passes of the
    construction tiles, 64-entry candidate lists): every tour a permutation
    with its exact length, sampled ants equal to the oracle's."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_1101_2678_amd.aco import Colony

    n, m = 4096, 64
    _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=4096)
    c = Colony(d, m, 1, 2, 0.5, 5, atomic=False)
    ch = c.choice()
    if rule == "nn":
        c.attach_nn(64)
        nnl = oracle.nn_lists(d, 64)
        assert (c.nn_lists() == nnl).all()
        c.construct_nn(0)
        ref = lambda k: oracle.construct_ant_nn(ch, d, nnl, 5, 0, k)
    elif rule == "product":
        c.construct_product(0)
        ref = lambda k: oracle.construct_ant_product(ch, d, 5, 0, k)
    else:
        c.construct(0)
        ref = lambda k: oracle.construct_ant(ch, d, 5, 0, k)
    tours, lens = c.tours()
    assert (np.sort(tours[:, :-1], axis=1) == np.arange(n, dtype=np.uint16)).all()
    t64 = tours.astype(np.int64)
    assert (d[t64[:, :-1], t64[:, 1:]].astype(np.int64).sum(axis=1) == lens).all()
    sample = [0, 1, 31, 63]
    log(f"  max cities rule={rule} ants {sample}")
    with ThreadPoolExecutor(ORACLE_THREADS) as ex:
        refs = list(ex.map(ref, sample))
    for k, (t, ln) in zip(sample, refs):
        assert (tours[k] == t).all() and lens[k] == ln, f"ant {k} differs"
    c.close()


def test_deposit_sums_at_the_exactness_bound():
    """The widest spread of tour lengths the library accepts at m = 65535:
    a ring of unit edges with chords of 3000 (every tour between 20 and
    60000, so 16 + 13 + 24 = 53 bits), where the deposit sums of a cell use
    nearly all 53 bits.  Every tour, length and tau bit-exact over 2
    iterations, all three updates (the gather and shared-memory ones sum in
    fixed point, the direct one in binary64)."""
    n = 20
    d = np.full((n, n), 3000, np.int32)
    for i in range(n):
        d[i, (i + 1) % n] = d[(i + 1) % n, i] = 1
    np.fill_diagonal(d, 0)
    ref = compare_run(d, 65535, 1, 2, 0.5, 11, iters=2,
                      kinds=("gather", "atomic", "atomic_direct"))
    assert ref.best_len >= n


def test_max_ants():
    """m = 65535 ants, the largest colony (one workgroup per ant, the top of
    the 16-bit ant field): every tour, length and tau bit-exact, all three
    updates (the shared-memory deposit splits the ants of a row over 128
    workgroups here)."""
    _, d = tsp_inputs.instance(16, "uniform", side=10_000, seed=65535)
    compare_run(d, 65535, 1, 2, 0.5, 7, iters=2, kinds=("gather", "atomic", "atomic_direct"))
