"""Pins for the CPU oracle: checks against things other than the oracle itself.

Every test here runs on the CPU.  Sources of truth: a third-party Philox
implementation (rocRAND, run, not copied), exact rational arithmetic,
closed forms, brute force on tiny instances, invariants of the update
(Eqs. 2-4), and chi-square tests of the sampled distribution against the
probabilities of Eq. (1).
"""
from __future__ import annotations

import itertools
import json
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import tsp_inputs

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "hand_values.json")))
U = Fraction(1, 2**24)  # unit roundoff of binary32


# ----------------------------------------------------------------- helpers
def nearest_f32(q: Fraction) -> np.float32:
    """Correctly rounded binary32 of a non-negative rational (ties to even),
    derived with exact integer arithmetic."""
    if q == 0:
        return np.float32(0.0)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    while Fraction(2) ** e > q:
        e -= 1
    while Fraction(2) ** (e + 1) <= q:
        e += 1
    scale = Fraction(2) ** (max(e, -126) - 23)
    N = q / scale
    fl = N.numerator // N.denominator
    rem = N - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return np.float32(float(fl * scale))


def f32bits(x) -> int:
    return int(np.asarray(x, np.float32).view(np.uint32))


def brute_force_opt(d: np.ndarray) -> int:
    n = d.shape[0]
    best = None
    for perm in itertools.permutations(range(1, n)):
        t = (0,) + perm + (0,)
        ln = sum(int(d[t[i], t[i + 1]]) for i in range(n))
        best = ln if best is None else min(best, ln)
    return best


def tour_length(d, tour) -> int:
    t = np.asarray(tour, np.int64)
    return int(d[t[:-1], t[1:]].astype(np.int64).sum())


# ----------------------------------------------------------------- inputs
def test_euc2d_hand_values():
    g = GOLD["euc2d_345"]
    assert tsp_inputs.euc2d(np.array(g["coords"])).tolist() == g["dist"]
    g = GOLD["euc2d_rounding"]
    d = tsp_inputs.euc2d(np.array(g["coords"]))
    assert (d[0, 1], d[0, 2], d[0, 3], d[0, 4]) == (g["d01"], g["d02"], g["d03"], g["d04"])


@pytest.mark.parametrize("layout", ["uniform", "cluster"])
def test_instances_distinct_symmetric(layout):
    xy, d = tsp_inputs.instance(300, layout, side=10_000, seed=3)
    assert len({tuple(p) for p in xy.tolist()}) == 300
    assert (d == d.T).all() and (np.diag(d) == 0).all()
    off = d[~np.eye(300, dtype=bool)]
    assert off.min() >= 1
    assert xy.min() >= 0 and xy.max() <= 10_000


def test_uniform_coordinates_chi2():
    """Uniform layout: per-axis and joint coordinate histograms are flat."""
    xy = tsp_inputs.uniform_cities(20000, 999, seed=7)
    for axis in (0, 1):
        counts = np.bincount(xy[:, axis] * 10 // 1000, minlength=10)
        assert stats.chisquare(counts).pvalue > 1e-4
    joint = np.bincount((xy[:, 0] * 8 // 1000) * 8 + xy[:, 1] * 8 // 1000, minlength=64)
    assert stats.chisquare(joint).pvalue > 1e-4


def test_cluster_sigma_estimate():
    """Clustered layout: 20 groups whose spread per axis is 2% of the side."""
    from sklearn.cluster import KMeans

    side = 1_000_000
    xy = tsp_inputs.clustered_cities(4000, side, seed=3).astype(np.float64)
    km = KMeans(n_clusters=20, n_init=10, random_state=0).fit(xy)
    spread = []
    for c in range(20):
        pts = xy[km.labels_ == c]
        if len(pts) > 50:
            spread.extend(np.std(pts, axis=0))
    assert 0.017 * side < np.median(spread) < 0.023 * side


def test_instance_fingerprints():
    """The seeded workloads are exactly those recorded (coordinates hashed)."""
    import hashlib

    want = json.load(open(os.path.join(HERE, "golden", "instance_hashes.json")))
    for key, digest in want.items():
        n, layout, side, seed = key.split("-")
        xy, _ = tsp_inputs.instance(int(n), layout, side=int(side), seed=int(seed))
        assert hashlib.sha256(xy.astype("<i8").tobytes()).hexdigest() == digest, key


# ----------------------------------------------------------------- Philox (C5)
def _rocrand_ref(tmp_path_factory, vectors):
    header = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(header) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    d = tmp_path_factory.mktemp("philox")
    exe = str(d / "ref")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe], check=True)
    inp = "\n".join(" ".join(f"{w:x}" for w in v) for v in vectors) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]


def test_philox_matches_rocrand(oracle_lib, tmp_path_factory):
    rng = np.random.default_rng(7)
    # rocRAND takes counter words 0-1 as offset*4 in 64 bits, so word 1 must stay
    # below 2^30 for the mapping to be exact (the AS puts the ant index there)
    vecs = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0x3FFFFFFF,
                                 0xFFFFFFFF, 0xFFFFFFFF]]
    r = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    r[:, 3] %= 2**30
    vecs += r.tolist()
    # the counters the AS actually uses: (step, ant, iter, 0), seed 1
    vecs += [[1, 0, s, k, it, 0] for s, k, it in [(0, 0, 0), (1, 0, 0), (4095, 65534, 7)]]
    ref = _rocrand_ref(tmp_path_factory, vecs)
    for v, r in zip(vecs, ref):
        key, ctr = v[:2], v[2:]
        got = oracle_lib.philox(ctr, key).tolist()
        assert got == r, (v, got, r)


def test_draw_keying(oracle_lib):
    # draw(seed, iter, ant, step) is word 0 of Philox(counter=(step, ant, iter, 0), key=seed)
    seed = 0x0123456789ABCDEF
    x = oracle_lib.draw(seed, 5, 17, 9)
    w = oracle_lib.philox([9, 17, 5, 0], [seed & 0xFFFFFFFF, seed >> 32])
    assert x == int(w[0])


def test_uniform_grid_and_range(oracle_lib):
    for x0 in [0, 255, 256, 0xFFFFFFFF, 0x80000000, 123456789]:
        u = oracle_lib.uniform(x0)
        assert Fraction(u) == Fraction(x0 >> 8, 2**24)
    assert oracle_lib.uniform(0xFFFFFFFF) == 1.0 - 2.0**-24


def test_start_city_uniform_chi2(oracle_lib):
    n = 7
    counts = np.zeros(n, np.int64)
    for k in range(20000):
        counts[oracle_lib.start_city(oracle_lib.draw(1, 0, k, 0), n)] += 1
    assert stats.chisquare(counts).pvalue > 1e-4
    # boundary: x0 = 2^32 - 1 maps to n - 1, x0 = 0 to 0
    assert oracle_lib.start_city(0xFFFFFFFF, 4096) == 4095
    assert oracle_lib.start_city(0, 4096) == 0


# ----------------------------------------------------------------- heuristic (C3)
def test_heur_hand_values(oracle_lib):
    for c in GOLD["heur"]["cases"]:
        assert f32bits(oracle_lib.heur(c["d"], c["beta"])) == int(c["bits"], 16), c


@pytest.mark.parametrize("beta", [1, 2, 3, 4])
def test_heur_exact_rational(oracle_lib, beta):
    rng = np.random.default_rng(beta)
    for d in rng.integers(1, 1_500_000, size=200).tolist() + [1, 2, 1_414_214]:
        h = oracle_lib.heur(d, beta)
        if beta <= 2:  # d^beta exact in binary64: one rounding to binary64, one to binary32
            q = Fraction(1, d**beta)
            # a binary64 quotient then a binary32 rounding is within 1 ulp32 of q
            assert abs(Fraction(float(h)) - q) <= q * 2 * U
        else:  # the binary64 power may round: still within a few ulps
            q = Fraction(1, d**beta)
            assert abs(Fraction(float(h)) - q) <= q * 4 * U


def test_choice_alpha_beta(oracle_lib):
    _, d = tsp_inputs.instance(20, "uniform", side=1000, seed=2)
    rng = np.random.default_rng(0)
    tau = rng.uniform(0.01, 2.0, size=(20, 20)).astype(np.float32)
    for alpha in (0, 1, 2):
        ch = oracle_lib.choice(tau, d, alpha, 2)
        assert (np.diag(ch) == 0).all()
        for i, j in [(0, 1), (3, 7), (19, 4)]:
            h = Fraction(float(oracle_lib.heur(int(d[i, j]), 2)))
            t = Fraction(float(tau[i, j]))
            tp = {0: Fraction(1), 1: t, 2: Fraction(float(nearest_f32(t * t)))}[alpha]
            assert f32bits(ch[i, j]) == f32bits(nearest_f32(tp * h))


# ----------------------------------------------------------------- tau0 (C4)
def test_nn_tour_collinear_closed_form(oracle_lib):
    g = GOLD["collinear_nn"]
    xy = np.array([[10 * i, 0] for i in range(g["n"])])
    d = tsp_inputs.euc2d(xy)
    assert oracle_lib.nn_tour_length(d) == g["c_nn"]
    st = oracle_lib.init(d, g["m"], 1, 2, 0.5, 1)
    assert f32bits(st.tau0) == int(g["tau0_bits"], 16)
    for n in (5, 17, 100):
        d = tsp_inputs.euc2d(np.array([[7 * i, 0] for i in range(n)]))
        assert oracle_lib.nn_tour_length(d) == 2 * 7 * (n - 1)


def test_nn_tour_ties_lowest_index(oracle_lib):
    # city 0 at the centre of a plus sign: four neighbours at equal distance
    xy = np.array([[5, 5], [5, 6], [4, 5], [6, 5], [5, 4]])
    d = tsp_inputs.euc2d(xy)
    # from 0 the tie (1,2,3,4 all at 1) goes to 1; from 1: 2 and 3 at nint(sqrt 2)=1 -> 2;
    # from 2: 4 at 1 (sqrt 2), 3 at 2 -> 4; from 4: 3 at 1 -> 3; back to 0: 1
    assert oracle_lib.nn_tour_length(d) == 1 + 1 + 1 + 1 + 1
    # a tie that changes the length: 0=(4,2) 1=(2,5) 2=(4,5) 3=(2,4) 4=(5,3).
    # 0->4 (nint sqrt 2 = 1), 4->2 (sqrt 5 -> 2), then 1 and 3 tie at 2 from
    # city 2: lowest index 1 (2), 1->3 (1), 3->0 (sqrt 8 -> 3): 9; taking 3
    # instead gives 3->1 (1), 1->0 (sqrt 13 -> 4): 10
    d = tsp_inputs.euc2d(np.array([[4, 2], [2, 5], [4, 5], [2, 4], [5, 3]]))
    assert oracle_lib.nn_tour_length(d) == 1 + 2 + 2 + 1 + 3


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_nn_tour_at_least_optimum(oracle_lib, seed):
    _, d = tsp_inputs.instance(8, "uniform", side=1000, seed=seed)
    assert oracle_lib.nn_tour_length(d) >= brute_force_opt(d)


# ----------------------------------------------------------------- S64 (C7)
def test_s64_integers_exact(oracle_lib):
    g = GOLD["s64_integers"]
    out = oracle_lib.s64(np.array(g["input"], np.float32))
    assert out.tolist() == np.cumsum(g["input"]).tolist()
    assert out[63] == g["last"]
    rng = np.random.default_rng(5)
    for _ in range(200):
        x = rng.integers(0, 1000, size=64) * (rng.random(64) < 0.6)
        assert oracle_lib.s64(x.astype(np.float32)).tolist() == np.cumsum(x).tolist()
    for _ in range(50):  # powers of two: also exact
        x = np.ldexp(1.0, rng.integers(-20, 0, size=64)).astype(np.float32)
        ex = np.cumsum([Fraction(float(v)) for v in x])
        assert [Fraction(float(v)) for v in oracle_lib.s64(x)] == list(ex)


def test_s64_association_hand_values(oracle_lib):
    """Which partial sums the tree adds in which order, pinned by a hand-derived
    example whose roundings tell the associations apart (the derivation is in
    the fixture's citation): entries 16..63 take the stage-B carries exactly as
    the tree defines them."""
    g = GOLD["s64_association"]
    out = oracle_lib.s64(np.array(g["input"], np.float32))
    assert [f32bits(v) for v in out] == [f32bits(v) for v in g["output"]]


def test_s64_total_is_pairwise_tree(oracle_lib):
    """Entry 63 of the tree is a balanced pairwise sum: ((x0+x1)+(x2+x3))+..."""
    rng = np.random.default_rng(11)
    for _ in range(500):
        x = (rng.random(64) * np.exp2(rng.integers(-30, 30, size=64))).astype(np.float32)
        x[rng.random(64) < 0.3] = 0
        y = x.copy()
        while y.size > 1:
            y = (y[0::2] + y[1::2]).astype(np.float32)
        assert f32bits(oracle_lib.s64(x)[63]) == f32bits(y[0])


def test_s64_error_bound(oracle_lib):
    """Every entry is within a depth-7 tree rounding bound of the exact prefix."""
    rng = np.random.default_rng(12)
    for _ in range(200):
        x = (rng.random(64) * np.exp2(rng.integers(-40, 20, size=64))).astype(np.float32)
        out = oracle_lib.s64(x)
        pref = Fraction(0)
        for t in range(64):
            pref += Fraction(float(x[t]))
            assert abs(Fraction(float(out[t])) - pref) <= pref * 7 * U * Fraction(101, 100)


# ----------------------------------------------------------------- R64 (C7)
def test_r64_single_feasible(oracle_lib):
    rng = np.random.default_rng(1)
    for n in (3, 64, 65, 130, 4096):
        row = rng.random(n).astype(np.float32)
        for j in (0, n // 2, n - 1):
            feas = np.zeros(n, np.uint8)
            feas[j] = 1
            for u in (0.0, 0.5, 1 - 2**-24):
                assert oracle_lib.r64_select(row, feas, u) == j


def test_r64_zero_total_takes_last_feasible(oracle_lib):
    n = 200
    row = np.zeros(n, np.float32)
    feas = np.zeros(n, np.uint8)
    feas[[3, 70, 150]] = 1
    assert oracle_lib.r64_select(row, feas, 0.3) == 150


def test_r64_u_zero_takes_first_positive(oracle_lib):
    rng = np.random.default_rng(2)
    for _ in range(100):
        n = int(rng.integers(3, 500))
        row = rng.random(n).astype(np.float32)
        row[rng.random(n) < 0.5] = 0
        feas = (rng.random(n) < 0.7).astype(np.uint8)
        pos = np.nonzero(feas.astype(bool) & (row > 0))[0]
        got = oracle_lib.r64_select(row, feas, 0.0)
        if pos.size:
            assert got == pos[0]
        else:
            assert got == np.nonzero(feas)[0][-1]


def test_r64_integer_weights_closed_form(oracle_lib):
    """Small integer weights make every sum exact, so R64 is the textbook
    inverse-CDF rule: the first j whose cumulative weight exceeds fl(u*total)."""
    rng = np.random.default_rng(3)
    for _ in range(400):
        n = int(rng.integers(3, 700))
        w = rng.integers(0, 50, size=n)
        feas = (rng.random(n) < 0.6).astype(np.uint8)
        if not feas.any():
            feas[n // 2] = 1
        wm = np.where(feas.astype(bool), w, 0)
        total = int(wm.sum())
        u = float(np.float32(int(rng.integers(0, 2**24)) / 2**24))
        target = Fraction(float(nearest_f32(Fraction(u) * total)))
        cum = np.cumsum(wm)
        cand = [j for j in range(n) if feas[j] and cum[j] > target]
        expect = cand[0] if cand else int(np.nonzero(feas)[0][-1])
        assert oracle_lib.r64_select(w.astype(np.float32), feas, u) == expect


def _eq1_probs(row, feas):
    w = np.where(np.asarray(feas, bool), np.asarray(row, np.float64), 0.0)
    return w / w.sum()


@pytest.mark.parametrize("n", [10, 150, 700])
def test_r64_stratified_matches_eq1(oracle_lib, n):
    """Eq. (1) exactly: u swept over an even grid of N points hits city j in
    N * p_j points, up to the FP32 rounding of the cumulative sums."""
    rng = np.random.default_rng(n)
    row = (rng.random(n) * np.exp2(rng.integers(-6, 2, size=n))).astype(np.float32)
    feas = (rng.random(n) < 0.8).astype(np.uint8)
    feas[0] = 1
    N = 1 << 14
    counts = np.zeros(n, np.int64)
    for k in range(N):
        counts[oracle_lib.r64_select(row, feas, (k * (2**24 // N)) / 2**24)] += 1
    p = _eq1_probs(row, feas)
    assert counts[feas == 0].sum() == 0
    # each boundary moves by at most a few binary32 ulps of the total
    assert np.abs(counts - N * p).max() <= 2


def _chi2_merged(counts, expected, min_exp=20.0):
    order = np.argsort(expected)
    obs_m, exp_m, acc_o, acc_e = [], [], 0, 0.0
    for i in order:
        acc_o += counts[i]
        acc_e += expected[i]
        if acc_e >= min_exp:
            obs_m.append(acc_o)
            exp_m.append(acc_e)
            acc_o, acc_e = 0, 0.0
    if acc_e > 0:
        obs_m[-1] += acc_o
        exp_m[-1] += acc_e
    return stats.chisquare(obs_m, exp_m).pvalue


@pytest.mark.parametrize("n,seed", [(10, 1), (150, 2)])
def test_r64_chi2_philox_draws(oracle_lib, n, seed):
    """End to end with the Philox draws of step 1: frequencies vs Eq. (1)."""
    rng = np.random.default_rng(n)
    row = (rng.random(n) * np.exp2(rng.integers(-6, 2, size=n))).astype(np.float32)
    feas = (rng.random(n) < 0.8).astype(np.uint8)
    feas[0] = 1
    draws = 40000
    counts = np.zeros(n, np.int64)
    for k in range(draws):
        counts[oracle_lib.r64_select(row, feas, oracle_lib.uniform(oracle_lib.draw(seed, 0, k, 1)))] += 1
    p = _eq1_probs(row, feas)
    idx = np.nonzero(feas)[0]
    assert counts[feas == 0].sum() == 0
    assert _chi2_merged(counts[idx], p[idx] * draws) > 1e-4


def test_r64_non_monotone_prefix_is_not_skipped(oracle_lib):
    """FP32 tree prefixes are not monotone: an inner entry can exceed the block
    total.  With the target at the total, the rule must still return the first
    feasible j whose prefix exceeds it (a block-first search would return the
    last feasible city instead)."""
    rng = np.random.default_rng(21)
    found = 0
    for _ in range(20000):
        w = rng.random(64).astype(np.float32)
        w[63] = 0.0
        s = oracle_lib.s64(w)
        if not (s[:63] > s[63]).any():
            continue
        u = 1.0 - 2.0**-24
        target = np.float32(np.float32(u) * s[63])
        over = np.nonzero(s > target)[0]
        if over.size == 0:
            continue
        feas = np.ones(64, np.uint8)
        assert oracle_lib.r64_select(w, feas, u) == over[0]
        assert over[0] < 63
        found += 1
        if found >= 5:
            break
    assert found >= 5


# ----------------------------------------------------------------- construction
@pytest.mark.parametrize("n,m", [(3, 4), (9, 9), (64, 10), (65, 7), (130, 5)])
def test_tours_are_permutations(oracle_lib, n, m):
    _, d = tsp_inputs.instance(n, "uniform", side=5000, seed=n)
    st = oracle_lib.init(d, m, 1, 2, 0.5, 1)
    tours, lens = oracle_lib.construct(st.choice, d, m, 1, 0)
    for k in range(m):
        t = tours[k]
        assert sorted(t[:-1].tolist()) == list(range(n))
        assert t[n] == t[0]
        assert t[0] == oracle_lib.start_city(oracle_lib.draw(1, 0, k, 0), n)
        assert lens[k] == tour_length(d, t)


def test_alpha_beta_zero_uniform_second_city(oracle_lib):
    """alpha = beta = 0 makes every unvisited city equally likely (Eq. 1)."""
    n = 6
    _, d = tsp_inputs.instance(n, "uniform", side=100, seed=4)
    st = oracle_lib.init(d, 1, 0, 0, 0.5, 1)
    counts = np.zeros((n, n), np.int64)
    tours, _ = oracle_lib.construct(st.choice, d, 12000, 5, 0)
    for t in tours:
        counts[t[0], t[1]] += 1
    for s in range(n):
        row = np.delete(counts[s], s)
        assert counts[s, s] == 0
        assert stats.chisquare(row).pvalue > 1e-4


# ----------------------------------------------------------------- nn-list construction
def _grid_instance(rows, cols, step=10):
    """Cities on an integer grid: many equal distances, so every tie rule
    is exercised."""
    xy = np.array([[step * c, step * r] for r in range(rows) for c in range(cols)], np.int64)
    return tsp_inputs.euc2d(xy)


@pytest.mark.parametrize("layout", ["uniform", "cluster", "grid"])
def test_nn_lists_match_lexsort(oracle_lib, layout):
    """Row i lists the nn nearest other cities by (d_ij, j), like a stable
    sort of the row by distance with city i removed."""
    if layout == "grid":
        d = _grid_instance(7, 9)
    else:
        _, d = tsp_inputs.instance(200, layout, side=3000, seed=8)
    n = d.shape[0]
    for nn in (1, 5, 30, n - 1):
        got = oracle_lib.nn_lists(d, nn)
        for i in range(n):
            others = np.delete(np.arange(n), i)
            order = others[np.lexsort((others, d[i, others]))]
            assert got[i].tolist() == order[:nn].tolist(), (layout, nn, i)


@pytest.mark.parametrize("n", [5, 64, 65, 130])
def test_nn_full_list_reduces_to_full_construction(oracle_lib, n):
    """With equal distances every list is 0..n-1 without i; with nn = n-1
    and integer weights (exact sums) the nn-list roulette then picks the
    same city as the roulette over the whole row, so the tours coincide
    with full construction.  The weights are not symmetric, so a
    transposed lookup would show."""
    d = np.full((n, n), 7, np.int32)
    np.fill_diagonal(d, 0)
    rng = np.random.default_rng(n)
    choice = rng.integers(0, 9, size=(n, n)).astype(np.float32)
    np.fill_diagonal(choice, 0)
    nnl = oracle_lib.nn_lists(d, n - 1)
    for i in range(n):
        assert nnl[i].tolist() == [j for j in range(n) if j != i]
    for k in range(40):
        t_nn, l_nn = oracle_lib.construct_ant_nn(choice, d, nnl, 3, 2, k)
        t_full, l_full = oracle_lib.construct_ant(choice, d, 3, 2, k)
        assert t_nn.tolist() == t_full.tolist() and l_nn == l_full


def _greedy_tour(d, start):
    """Textbook nearest-neighbour tour: always the closest unvisited city,
    the lowest index among equally close ones."""
    n = d.shape[0]
    seen = [False] * n
    tour = [start]
    seen[start] = True
    for _ in range(n - 1):
        cur = tour[-1]
        nxt = min((j for j in range(n) if not seen[j]), key=lambda j: (d[cur, j], j))
        tour.append(nxt)
        seen[nxt] = True
    return tour + [start]


@pytest.mark.parametrize("case", ["uniform", "grid"])
def test_nn_one_with_decreasing_choice_is_greedy_tour(oracle_lib, case):
    """nn = 1 and choice strictly decreasing in d: the listed neighbour is
    the nearest city, and the fallback (largest choice among the unvisited)
    is the nearest unvisited city, so every tour is the nearest-neighbour
    tour from its start city."""
    if case == "grid":
        d = _grid_instance(5, 6)
    else:
        _, d = tsp_inputs.instance(60, "uniform", side=100_000, seed=5)
    n = d.shape[0]
    with np.errstate(divide="ignore"):
        choice = (1.0 / (d.astype(np.float64) ** 2)).astype(np.float32)
    np.fill_diagonal(choice, 0)
    nnl = oracle_lib.nn_lists(d, 1)
    for k in range(25):
        t, ln = oracle_lib.construct_ant_nn(choice, d, nnl, 11, 0, k)
        start = oracle_lib.start_city(oracle_lib.draw(11, 0, k, 0), n)
        want = _greedy_tour(d, start)
        assert t.tolist() == want
        assert ln == tour_length(d, want)


def test_nn_fallback_takes_largest_choice_lowest_index(oracle_lib):
    """Once the listed neighbours are visited the ant goes to the unvisited
    city with the largest choice value; equal values go to the lowest
    index.  Choice values here are chosen so that this city is never the
    nearest one."""
    n = 12
    _, d = tsp_inputs.instance(n, "uniform", side=1000, seed=3)
    nnl = oracle_lib.nn_lists(d, 1)
    # choice[i][j] = j mod 4 (ties in groups): the argmax over unvisited j is
    # the lowest unvisited j with the largest residue
    choice = np.tile((np.arange(n) % 4).astype(np.float32), (n, 1))
    np.fill_diagonal(choice, 0)
    for k in range(30):
        t, _ = oracle_lib.construct_ant_nn(choice, d, nnl, 4, 1, k)
        seen = {int(t[0])}
        for s in range(1, n):
            cur = int(t[s - 1])
            nb = int(nnl[cur, 0])
            unv = [j for j in range(n) if j not in seen]
            if nb not in seen:
                want = nb
            else:
                best = max(choice[cur, j] for j in unv)
                want = min(j for j in unv if choice[cur, j] == best)
            assert int(t[s]) == want, (k, s)
            seen.add(want)


@pytest.mark.parametrize("seed", [1, 2])
def test_nn_second_city_follows_eq1_on_the_list(oracle_lib, seed):
    """At step 1 only the start is visited and it is on no list of its
    own, so the second city is drawn from the start's list with
    probabilities choice / (sum over the list): Eq. (1) restricted to the
    candidate list."""
    n, nn, ants = 7, 3, 21000
    _, d = tsp_inputs.instance(n, "uniform", side=1000, seed=6)
    st = oracle_lib.init(d, 7, 1, 2, 0.5, 1)
    nnl = oracle_lib.nn_lists(d, nn)
    tours, _ = oracle_lib.construct_nn(st.choice, d, nnl, ants, seed, 0, threads=4)
    for s in range(n):
        sec = tours[tours[:, 0] == s, 1]
        assert set(sec.tolist()) <= set(nnl[s].tolist())
        w = st.choice[s, nnl[s]].astype(np.float64)
        obs = np.array([(sec == c).sum() for c in nnl[s]])
        assert stats.chisquare(obs, w / w.sum() * obs.sum()).pvalue > 1e-4


@pytest.mark.parametrize("n,nn", [(3, 1), (3, 2), (40, 5), (130, 30), (257, 64)])
def test_nn_tours_are_permutations(oracle_lib, n, nn):
    _, d = tsp_inputs.instance(n, "cluster", side=20_000, seed=n)
    st = oracle_lib.init(d, 8, 1, 2, 0.5, 2)
    nnl = oracle_lib.nn_lists(d, nn)
    tours, lens = oracle_lib.construct_nn(st.choice, d, nnl, 8, 2, 0)
    for k in range(8):
        t = tours[k]
        assert sorted(t[:-1].tolist()) == list(range(n)) and t[n] == t[0]
        assert t[0] == oracle_lib.start_city(oracle_lib.draw(2, 0, k, 0), n)
        assert lens[k] == tour_length(d, t)


# ----------------------------------------------------------------- product-and-argmax rule
def test_product_uniform_matches_rocrand(oracle_lib, tmp_path_factory):
    """r_j is word j mod 4 of Philox at counter (step, ant, iter, 1 + j / 4),
    checked against rocRAND's own engine (run, not copied)."""
    cases = [(1, 0, 0, 1, 0), (1, 0, 0, 1, 3), (7, 3, 11, 5, 4), (2**40 + 5, 9, 65534, 4095, 4095),
             (3, 2, 1, 7, 2398), (3, 2, 1, 7, 2399), (99, 1, 2, 3, 17)]
    vecs = [[seed & 0xFFFFFFFF, seed >> 32, step, ant, it, 1 + j // 4]
            for seed, it, ant, step, j in cases]
    ref = _rocrand_ref(tmp_path_factory, vecs)
    for (seed, it, ant, step, j), words in zip(cases, ref):
        want = (words[j % 4] >> 8) * 2.0**-24
        assert oracle_lib.product_uniform(seed, it, ant, step, j) == want


def test_product_select_ties_exclusions_rounding(oracle_lib):
    sel = oracle_lib.product_select
    f32 = lambda *v: np.array(v, np.float32)
    # equal products: the lowest index
    assert sel(f32(2, 1), [1, 1], f32(0.25, 0.5)) == 0
    assert sel(f32(1, 2, 1), [0, 1, 1], f32(0.5, 0.25, 0.5)) == 1
    # a visited city never wins, however large its product
    assert sel(f32(100, 1, 2), [0, 1, 1], f32(0.9, 0.1, 0.01)) == 1
    # all feasible products zero: the lowest feasible city
    assert sel(f32(5, 0, 3, 0), [0, 1, 1, 1], f32(0.5, 0.5, 0.0, 0.5)) == 1
    assert sel(f32(1, 1), [0, 0], f32(0.5, 0.5)) == -1
    # the comparison is on binary32 products: exact products that differ but
    # round to the same binary32 value tie, and the lowest index wins
    w0, r0 = 1.0 + 2.0**-23, 1.0 - 2.0**-23          # exact product 1 - 2^-46
    w1, r1 = 1.0 + 2.0**-23, 1.0 - 2.0**-24          # exact product 1 + 2^-24 - 2^-47
    p0 = nearest_f32(Fraction(w0) * Fraction(r0))
    p1 = nearest_f32(Fraction(w1) * Fraction(r1))
    assert Fraction(w0) * Fraction(r0) < Fraction(w1) * Fraction(r1)
    assert p0 == p1
    assert sel(f32(w0, w1), [1, 1], f32(r0, r1)) == 0
    assert sel(f32(w1, w0), [1, 1], f32(r1, r0)) == 0


def _argmax_win_probabilities(w):
    """P(j has the largest w_j r_j) for independent uniform r: the integral
    over x of prod_{k != j} min(1, w_j x / w_k)."""
    from scipy import integrate

    w = np.asarray(w, np.float64)
    probs = []
    for j in range(len(w)):
        f = lambda x: np.prod([min(1.0, w[j] * x / w[k]) for k in range(len(w)) if k != j])
        pts = sorted({min(1.0, w[k] / w[j]) for k in range(len(w)) if k != j})
        probs.append(integrate.quad(f, 0.0, 1.0, points=pts, limit=200)[0])
    return np.array(probs)


def test_product_win_probabilities_two_cities(oracle_lib):
    """n = 3: after the start, two cities remain and the one with weight a
    beats weight b >= a with probability a / (2 b)."""
    choice = np.array([[0, 1, 3], [2, 0, 5], [4, 4, 0]], np.float32)
    d = np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], np.int32)
    tours, _ = oracle_lib.construct_product(choice, d, 30000, 5, 0, threads=4)
    for s, (a, b) in [(0, (1, 2)), (1, (0, 2)), (2, (0, 1))]:
        sec = tours[tours[:, 0] == s, 1]
        wa, wb = float(choice[s, a]), float(choice[s, b])
        pa = wa / (2 * wb) if wa <= wb else 1 - wb / (2 * wa)
        k = int((sec == a).sum())
        assert stats.binomtest(k, len(sec), pa).pvalue > 1e-4, (s, k, len(sec), pa)


@pytest.mark.parametrize("seed", [1, 2])
def test_product_win_probabilities_many_cities(oracle_lib, seed):
    """Second-city frequencies against the exact argmax probabilities; they
    differ from Eq. (1)'s proportional ones, which the test also shows."""
    n = 6
    rng = np.random.default_rng(seed)
    choice = rng.integers(1, 9, size=(n, n)).astype(np.float32)
    np.fill_diagonal(choice, 0)
    d = np.ones((n, n), np.int32)
    np.fill_diagonal(d, 0)
    tours, _ = oracle_lib.construct_product(choice, d, 36000, seed, 0, threads=4)
    far_from_eq1 = 0
    for s in range(n):
        others = [j for j in range(n) if j != s]
        p = _argmax_win_probabilities(choice[s, others])
        sec = tours[tours[:, 0] == s, 1]
        obs = np.array([(sec == j).sum() for j in others])
        assert abs(p.sum() - 1.0) < 1e-9
        assert stats.chisquare(obs, p / p.sum() * obs.sum()).pvalue > 1e-4, s
        q = choice[s, others].astype(np.float64) / choice[s, others].astype(np.float64).sum()
        far_from_eq1 += stats.chisquare(obs, q * obs.sum()).pvalue < 1e-6
    assert far_from_eq1 >= 4


def test_product_alpha_beta_zero_uniform_second_city(oracle_lib):
    """alpha = beta = 0: every product is a plain uniform, so every
    unvisited city is equally likely."""
    n = 6
    _, d = tsp_inputs.instance(n, "uniform", side=100, seed=4)
    st = oracle_lib.init(d, 1, 0, 0, 0.5, 1)
    tours, _ = oracle_lib.construct_product(st.choice, d, 12000, 5, 0, threads=4)
    counts = np.zeros((n, n), np.int64)
    for t in tours:
        counts[t[0], t[1]] += 1
    for s in range(n):
        assert counts[s, s] == 0
        assert stats.chisquare(np.delete(counts[s], s)).pvalue > 1e-4


@pytest.mark.parametrize("n,m", [(3, 4), (9, 9), (64, 10), (65, 7), (130, 5)])
def test_product_tours_are_permutations(oracle_lib, n, m):
    _, d = tsp_inputs.instance(n, "cluster", side=5000, seed=n)
    st = oracle_lib.init(d, m, 1, 2, 0.5, 3)
    tours, lens = oracle_lib.construct_product(st.choice, d, m, 3, 1)
    for k in range(m):
        t = tours[k]
        assert sorted(t[:-1].tolist()) == list(range(n)) and t[n] == t[0]
        assert t[0] == oracle_lib.start_city(oracle_lib.draw(3, 1, k, 0), n)
        assert lens[k] == tour_length(d, t)


# ----------------------------------------------------------------- update (C9-C11)
def test_evaporation_closed_form(oracle_lib):
    """Cells no tour touches follow tau0 * (1 - rho)^k (Eq. 2)."""
    n = 12
    _, d = tsp_inputs.instance(n, "uniform", side=1000, seed=6)
    st = oracle_lib.init(d, 1, 1, 2, 0.5, 1)
    tour = np.array([list(range(n)) + [0]], np.uint16)  # only edges {i, i+1}
    lens = np.array([tour_length(d, tour[0])], np.int64)
    onring = np.zeros((n, n), bool)
    for i in range(n):
        onring[i, (i + 1) % n] = onring[(i + 1) % n, i] = True
    tau = st.tau
    t0 = Fraction(float(st.tau0))
    for k in range(1, 31):
        tau, _ = oracle_lib.update(tau, tour, lens, d, 0.5, 1, 2)
        want = nearest_f32(t0 * Fraction(1, 2) ** k)  # exact: power-of-two scaling
        assert (tau[~onring].view(np.uint32) == f32bits(want)).all()
    # rho = 0.3: within 2k ulps of the exact power
    tau = st.tau
    for k in range(1, 21):
        tau, _ = oracle_lib.update(tau, tour, lens, d, 0.3, 1, 2)
        exact = t0 * Fraction(7, 10) ** k
        got = Fraction(float(tau[0, 5]))
        assert abs(got - exact) <= exact * 2 * k * U


def test_choice_refreshed_after_update(oracle_lib):
    """With beta = 0 the heuristic is 1 off the diagonal, so after every
    update choice must equal tau' bit for bit (alpha = 1), or the correctly
    rounded tau'^2 (alpha = 2); the diagonal stays 0."""
    n = 11
    _, d = tsp_inputs.instance(n, "uniform", side=1000, seed=12)
    off = ~np.eye(n, dtype=bool)
    for alpha in (1, 2):
        st = oracle_lib.init(d, 3, alpha, 0, 0.5, 4)
        tau = st.tau
        for it in range(3):
            tours, lens = oracle_lib.construct(st.choice if it == 0 else ch, d, 3, 4, it)
            tau, ch = oracle_lib.update(tau, tours, lens, d, 0.3, alpha, 0)
            assert (np.diag(ch) == 0).all()
            if alpha == 1:
                assert (ch[off].view(np.uint32) == tau[off].view(np.uint32)).all()
            else:
                for i, j in [(0, 1), (4, 9), (10, 2)]:
                    t = Fraction(float(tau[i, j]))
                    assert f32bits(ch[i, j]) == f32bits(nearest_f32(t * t))


def test_deposit_amount_large_lengths(oracle_lib):
    """dep = fl32(1 / (double) C^k) (Eq. 4, Q = 1) for tour lengths beyond
    2^24, where a binary32 length would already be rounded (real lengths at
    n = 2400 in a 10^6 square are ~5 * 10^7).  Python's division is IEEE
    binary64; the binary32 rounding is done exactly."""
    for L in [1, 3, 7, 2**24 - 1, 2**24 + 1, 2**24 + 3, 50_000_003, 123_456_789,
              1_234_567_891, 2**31 + 11, 4_200_000_001, 2**40 + 1]:
        want = nearest_f32(Fraction(1.0 / L))
        assert f32bits(oracle_lib.deposit_amount(L)) == f32bits(want), L


def test_deposit_exact_against_fractions(oracle_lib):
    """D_ij equals the exact rational sum of 1/C^k deposits (rounded to binary32
    per ant) over ants using edge {i,j}; sum_{i<j} D = n * sum_k dep_k."""
    n, m = 9, 13
    _, d = tsp_inputs.instance(n, "uniform", side=1000, seed=8)
    st = oracle_lib.init(d, m, 1, 2, 0.5, 1)
    tours, lens = oracle_lib.construct(st.choice, d, m, 3, 0)
    D, status = oracle_lib.deposit(tours, lens, n)
    assert status == 0
    dep = [Fraction(float(nearest_f32(Fraction(1, int(L))))) for L in lens]
    exact = [[Fraction(0)] * n for _ in range(n)]
    for k in range(m):
        t = tours[k]
        for s in range(n):
            i, j = int(t[s]), int(t[s + 1])
            exact[i][j] += dep[k]
            exact[j][i] += dep[k]
    for i in range(n):
        for j in range(n):
            assert Fraction(float(D[i, j])) == exact[i][j]
    upper = sum(Fraction(float(D[i, j])) for i in range(n) for j in range(i + 1, n))
    assert upper == n * sum(dep)


@pytest.mark.parametrize("rho", [0.5, 0.3])
def test_update_single_rounding_against_fractions(oracle_lib, rho):
    """tau' = fl32(fl32(tau * fl32(1 - rho)) + D) with D the exact sum of the
    deposits on the edge (Eqs. 2-3): every cell against exact rationals, one
    rounding after the sum, over three iterations of a 13-ant colony."""
    n, m = 9, 13
    _, d = tsp_inputs.instance(n, "uniform", side=1000, seed=8)
    st = oracle_lib.init(d, m, 1, 2, rho, 1)
    keep = Fraction(float(nearest_f32(1 - Fraction(float(np.float32(rho))))))
    tau, ch = st.tau, st.choice
    for it in range(3):
        tours, lens = oracle_lib.construct(ch, d, m, 3, it)
        dep = [Fraction(float(nearest_f32(Fraction(1, int(L))))) for L in lens]
        D = [[Fraction(0)] * n for _ in range(n)]
        for k in range(m):
            t = tours[k]
            for s in range(n):
                i, j = int(t[s]), int(t[s + 1])
                D[i][j] += dep[k]
                D[j][i] += dep[k]
        new_tau, ch = oracle_lib.update(tau, tours, lens, d, rho, 1, 2)
        for i in range(n):
            for j in range(n):
                a = Fraction(float(nearest_f32(Fraction(float(tau[i, j])) * keep)))
                assert f32bits(new_tau[i, j]) == f32bits(nearest_f32(a + D[i][j])), (it, i, j)
        tau = new_tau


def test_deposit_invariant_large(oracle_lib):
    n, m = 300, 300
    _, d = tsp_inputs.instance(n, "cluster", side=1_000_000, seed=9)
    st = oracle_lib.init(d, m, 1, 2, 0.5, 1)
    tours, lens = oracle_lib.construct(st.choice, d, m, 1, 0)
    D, status = oracle_lib.deposit(tours, lens, n)
    assert status == 0
    dep = sum(Fraction(float(oracle_lib.deposit_amount(int(L)))) for L in lens)
    iu = np.triu_indices(n, 1)
    assert sum(Fraction(float(v)) for v in D[iu]) == n * dep
    assert (D == D.T).all()
    # the new tau is symmetric bit for bit
    tau, _ = oracle_lib.update(st.tau, tours, lens, d, 0.5, 1, 2)
    assert (tau.view(np.uint32) == tau.T.view(np.uint32)).all()


def test_single_ant_full_evaporation(oracle_lib):
    """m = 1, rho = 1: tau' = dep_0 on exactly the 2n cells of the tour."""
    n = 40
    _, d = tsp_inputs.instance(n, "uniform", side=1000, seed=10)
    st = oracle_lib.init(d, 1, 1, 2, 1.0, 1)
    tours, lens = oracle_lib.construct(st.choice, d, 1, 1, 0)
    tau, _ = oracle_lib.update(st.tau, tours, lens, d, 1.0, 1, 2)
    dep = oracle_lib.deposit_amount(int(lens[0]))
    assert f32bits(dep) == f32bits(nearest_f32(Fraction(1, int(lens[0]))))
    nz = np.argwhere(tau != 0)
    assert len(nz) == 2 * n
    assert (tau[tau != 0] == dep).all()


# ----------------------------------------------------------------- whole solve
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_solve_small_reaches_optimum(oracle_lib, seed):
    """n = 8: every tour is at least the brute-force optimum (a theorem), and
    the best-so-far ends within 5% of it (a sanity bound only: AS with
    rho = 0.5 can stagnate, so optimality is not guaranteed)."""
    _, d = tsp_inputs.instance(8, "uniform", side=1000, seed=seed)
    opt = brute_force_opt(d)
    st = oracle_lib.init(d, 8, 1, 2, 0.5, seed)
    for _ in range(20):
        tours, lens = oracle_lib.iterate(st, d)
        assert (lens >= opt).all()
    assert opt <= st.best_len <= 1.05 * opt
    assert tour_length(d, st.best_tour) == st.best_len


def test_solve_deterministic_and_resumable(oracle_lib):
    _, d = tsp_inputs.instance(50, "uniform", side=1000, seed=12)
    a = oracle_lib.solve(d, 30, 1, 2, 0.5, 7, 6)
    b = oracle_lib.init(d, 30, 1, 2, 0.5, 7)
    for _ in range(3):
        oracle_lib.iterate(b, d)
    # resume from the saved tau/choice/iteration of b
    c = oracle_lib.init(d, 30, 1, 2, 0.5, 7)
    c.tau, c.choice, c.it, c.best_len = b.tau.copy(), b.choice.copy(), b.it, b.best_len
    c.best_tour = b.best_tour
    for _ in range(3):
        oracle_lib.iterate(c, d)
    assert (a.tau.view(np.uint32) == c.tau.view(np.uint32)).all()
    assert a.best_len == c.best_len


def test_best_of_strict_and_earliest(oracle_lib):
    """Best-so-far: the shortest length wins, the lowest ant index among equal
    lengths, and it replaces the stored best only if strictly shorter."""
    import ctypes

    lens = np.array([50, 40, 40, 45, 40], np.int64)
    best = ctypes.c_int64(2**62)
    assert oracle_lib.lib().oracle_best_of(5, lens, ctypes.byref(best)) == 1
    assert best.value == 40
    best = ctypes.c_int64(40)
    assert oracle_lib.lib().oracle_best_of(5, lens, ctypes.byref(best)) == -1
    best = ctypes.c_int64(41)
    assert oracle_lib.lib().oracle_best_of(5, lens, ctypes.byref(best)) == 1


# ----------------------------------------------------------------- arithmetic environment (C14)
def test_build_flags_fix_the_arithmetic():
    """Both sides are compiled without FP contraction and without fast-math;
    the GPU side also keeps binary32 subnormals and avoids packed FP32."""
    from paper_1101_2678_amd import _build

    flags = " ".join(_build.HIP_FLAGS)
    assert "-ffp-contract=off" in flags
    assert "-fno-gpu-flush-denormals-to-zero" in flags
    assert "-packed-fp32-ops" in flags and "-ffast-math" not in flags
    src = open(os.path.join(os.path.dirname(HERE), "oracle", "__init__.py")).read()
    assert "-ffp-contract=off" in src and "-ffast-math" not in src


def test_oracle_does_not_depend_on_contraction(oracle_lib, tmp_path):
    """The oracle has no same-precision a*b + c: built with contraction and
    FMA instructions allowed it gives the same bits for construction and
    update (so its pins do not hinge on the compiler flag)."""
    import ctypes

    cpu = open("/proc/cpuinfo").read() if os.path.exists("/proc/cpuinfo") else ""
    if shutil.which("gcc") is None or " fma" not in cpu:
        pytest.skip("gcc or an FMA-capable host CPU not available")
    src = os.path.join(os.path.dirname(HERE), "oracle", "aco_oracle.c")
    so = str(tmp_path / "liboracle_contract.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=fast", "-mfma", "-fPIC", "-shared",
                    src, "-o", so, "-lm"], check=True)
    alt = ctypes.CDLL(so)
    n, m = 60, 40
    _, d = tsp_inputs.instance(n, "uniform", side=100_000, seed=12)
    st = oracle_lib.init(d, m, 2, 3, 0.3, 9)
    tours, lens = oracle_lib.construct(st.choice, d, m, 9, 0)
    tau_ref, ch_ref = oracle_lib.update(st.tau, tours, lens, d, 0.3, 2, 3)
    f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    alt.oracle_update.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                  np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS"),
                                  np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS"),
                                  np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"),
                                  ctypes.c_int32, ctypes.c_int32, f32p, f32p]
    alt.oracle_update.restype = ctypes.c_int32
    tau_alt = st.tau.copy()
    ch_alt = np.empty_like(ch_ref)
    assert alt.oracle_update(n, m, np.float32(0.3), tours, lens, np.ascontiguousarray(d, np.int32),
                             2, 3, tau_alt, ch_alt) == 0
    assert (tau_alt.view(np.uint32) == tau_ref.view(np.uint32)).all()
    assert (ch_alt.view(np.uint32) == ch_ref.view(np.uint32)).all()
    alt.oracle_construct_ant.argtypes = [ctypes.c_int32, f32p,
                                         np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS"),
                                         ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                         np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")]
    alt.oracle_construct_ant.restype = ctypes.c_int64
    for k in range(5):
        t = np.empty(n + 1, np.uint16)
        ln = alt.oracle_construct_ant(n, st.choice, np.ascontiguousarray(d, np.int32), 9, 0, k, t)
        assert ln == lens[k] and (t == tours[k]).all()
