"""GPU: aco_update_atomic_noalloc, the atomic update whose binary64 deposit
matrix is the library's static device array, gives the same bits as
aco_update(ACO_UPDATE_ATOMIC) with the workspace's matrix: two calls in a row
on one GPU, the second on a smaller instance (the array keeps what the first
left), then the size limit and the call order."""
from __future__ import annotations

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
    torch.cuda.init()


def _run_pair(n, m, seed, iters):
    """A context without the atomic workspace part updated by the static
    variant, beside one with it updated by aco_update(ATOMIC): tours,
    lengths, tau and choice identical after every iteration."""
    from paper_1101_2678_amd.aco import Colony

    log(f"  noalloc n={n} m={m} seed={seed} iters={iters}")
    _, d = tsp_inputs.instance(n, "uniform", side=1_000_000, seed=seed)
    static = Colony(d, m, 1, 2, 0.5, seed, atomic=False)
    ref = Colony(d, m, 1, 2, 0.5, seed, atomic=True)
    for it in range(iters):
        static.construct(it)
        ref.construct(it)
        st, sl = static.tours()
        rt, rl = ref.tours()
        assert (st == rt).all() and (sl == rl).all(), f"it={it}: tours differ"
        static.update_atomic_noalloc()
        ref.update("atomic")
        assert_same_f32(static.tau(), ref.tau(), f"n={n} it={it} tau")
        assert_same_f32(static.choice(), ref.choice(), f"n={n} it={it} choice")
    assert static.best()[1] == ref.best()[1]
    static.close()
    ref.close()


def test_noalloc_matches_atomic_two_calls_second_smaller():
    _run_pair(1000, 300, 11, 3)   # 1000 x 1024 cells: close to the array's limit
    _run_pair(150, 60, 12, 3)     # smaller instance on the same array


def test_noalloc_refuses_above_limit_and_out_of_order():
    from paper_1101_2678_amd.aco import ACO_ERR_INVALID, ACO_ERR_STATE, AcoError, Colony

    _, d = tsp_inputs.instance(1025, "uniform", side=1_000_000, seed=3)
    big = Colony(d, 8, 1, 2, 0.5, 3, atomic=False)
    big.construct(0)
    with pytest.raises(AcoError) as e:
        big.update_atomic_noalloc()
    assert e.value.status == ACO_ERR_INVALID
    big.update("gather")          # the refused call left the pending construction
    big.sync()
    big.close()
    _, d = tsp_inputs.instance(64, "uniform", side=10_000, seed=4)
    small = Colony(d, 16, 1, 2, 0.5, 4, atomic=False)
    with pytest.raises(AcoError) as e:
        small.update_atomic_noalloc()
    assert e.value.status == ACO_ERR_STATE
    tau0 = small.tau()
    small.construct(0)
    small.update_atomic_noalloc()
    assert not np.array_equal(small.tau(), tau0)
    small.close()
