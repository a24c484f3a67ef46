"""GPU: seeded random configurations across every rule and update variant.

Each case draws n, m, alpha, beta, rho, the layout, the Philox seed and the
construction rule (and the list length for candidate lists) from a fixed
seed; every tour, length, tau and choice must equal the oracle's over two
iterations, for both update variants.
"""
from __future__ import annotations

import numpy as np
import pytest

import tsp_inputs
from gpu_helpers import compare_run

pytestmark = pytest.mark.gpu

RULES = ("r64", "nn", "product")


def _case(q: int):
    rng = np.random.default_rng([2026, q])
    n = int(np.exp(rng.uniform(np.log(3), np.log(700))))
    m = int(rng.integers(1, 200))
    alpha = int(rng.integers(0, 3))
    beta = int(rng.integers(0, 5))
    rho = float(np.float32(rng.choice([0.1, 0.25, 0.5, 0.75, 1.0, rng.uniform(0.01, 1.0)])))
    layout = "cluster" if rng.random() < 0.5 else "uniform"
    seed = int(rng.integers(1, 2**40))
    rule = RULES[q % 3]
    nn = int(rng.integers(1, min(64, n - 1) + 1)) if rule == "nn" else None
    side = int(rng.choice([1000, 100_000, 1_000_000]))
    side = max(side, 4 * n)  # room for n distinct integer points
    return n, m, alpha, beta, rho, layout, seed, rule, nn, side


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("q", range(16))
def test_random_config(q):
    n, m, alpha, beta, rho, layout, seed, rule, nn, side = _case(q)
    _, d = tsp_inputs.instance(n, layout, side=side, seed=seed % 100_000)
    compare_run(d, m, alpha, beta, rho, seed, iters=2, nn=nn, rule=rule)
