"""Construction with several wavefronts per ant (rows of at most 1024 cities):
the selection, the tours, lengths, tau and choice must equal the oracle's bit
for bit whatever the shape, since the block totals, the block bound and the
rescan are those of the single-wave kernel (Section II, Eq. 1; the ant's
cities spread over the threads of its block, Section III-A)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import tsp_inputs
from gpu_helpers import compare_run, log
from test_gpu_parity import _adversarial_rows

pytestmark = pytest.mark.gpu

SPLIT = ((8, 2), (4, 2), (4, 4))


def split_shapes(n):
    """The multi-wave shapes the library accepts for n (its documented rule:
    n <= 1024, at least as many passes of 64 * tile cities as waves, tile 8
    only with 2 waves, 4 waves only at 4 passes)."""
    out = []
    for tile, waves in SPLIT:
        passes = -(-n // (64 * tile))
        if n > 1024 or waves > passes:
            continue
        if waves == 4 and passes != 4:
            continue
        out.append((tile, waves))
    return out


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


@pytest.fixture
def shape_table():
    from paper_1101_2678_amd import aco

    aco.reset_tiles()
    yield aco
    aco.reset_tiles()


def test_shape_table_rule(shape_table):
    """aco_set_shape accepts exactly the shapes of the documented rule."""
    aco = shape_table
    for n in (1, 100, 256, 257, 512, 513, 768, 769, 1000, 1024, 1025, 2400):
        for tile, waves in SPLIT:
            ok = (tile, waves) in split_shapes(n)
            try:
                aco.set_shape(n, n, tile, waves)
                accepted = True
            except Exception:
                accepted = False
            assert accepted == ok, (n, tile, waves)
            if accepted:
                assert aco.get_tile(n) == tile and aco.get_waves(n) == waves
    with pytest.raises(Exception):
        aco.set_shape(600, 1024, 4, 4)  # 600..768 have three passes of 256
    aco.reset_tiles()
    assert all(aco.get_waves(n) == 1 for n in (3, 500, 1000, 4096))


@pytest.mark.parametrize("n", [257, 300, 511, 512, 513, 640, 768, 769, 1000, 1023, 1024])
def test_select_adversarial_split(n):
    import torch
    from paper_1101_2678_amd import aco

    rng = np.random.default_rng(5000 + n)
    count = 3000
    rows, feas, u = _adversarial_rows(n, count, rng)
    want = oracle.r64_select_batch(rows, feas, u)
    r, f, uu = (torch.from_numpy(x).cuda() for x in (rows, feas, u))
    for tile, waves in split_shapes(n):
        log(f"  select n={n} tile={tile} waves={waves} count={count}")
        got = aco.test_select(r, f, uu, tile=tile, waves=waves).cpu().numpy()
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"tile {tile} waves {waves}: {bad.size} rows differ, first {bad[:5]}"


@pytest.mark.parametrize("n,m,alpha,beta,rho", [
    (257, 40, 1, 2, 0.5), (300, 33, 2, 1, 0.3), (513, 64, 1, 2, 0.5), (600, 50, 1, 3, 0.9),
    (769, 31, 1, 2, 0.5), (1000, 70, 0, 2, 0.5), (1024, 64, 1, 2, 0.2),
])
def test_parity_split_ragged(shape_table, n, m, alpha, beta, rho):
    """Every multi-wave shape of n: tours, lengths, tau and choice of 3
    iterations bit-exact against the oracle, both update variants."""
    aco = shape_table
    _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=n + 11)
    for tile, waves in split_shapes(n):
        aco.set_shape(n, n, tile, waves)
        log(f"  shape tile={tile} waves={waves}")
        compare_run(d, m, alpha, beta, rho, seed=n + 5, iters=3)
    aco.reset_tiles()


@pytest.mark.parametrize("tile,waves", [(8, 2), (4, 4)])
def test_parity_n1000_split(shape_table, tile, waves):
    """The n = m = 1000 workload (uniform, instance seed 1, alpha 1, beta 2,
    rho 0.5, Philox seed 1) through a multi-wave shape: 5 iterations of
    tours, lengths, tau and choice bit-exact against the oracle."""
    from paper_1101_2678_amd.aco import Colony

    aco = shape_table
    aco.set_shape(1000, 1000, tile, waves)
    _, d = tsp_inputs.instance(1000, "uniform", side=1_000_000, seed=1)
    c = Colony(d, 1000, 1, 2, 0.5, 1)
    assert f"waves_per_ant={waves} cities_per_lane={tile}" in c.describe()
    c.close()
    compare_run(d, 1000, 1, 2, 0.5, 1, 5)
