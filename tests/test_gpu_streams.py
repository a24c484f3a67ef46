"""GPU: device memory handed to the library stays reserved while work queued
on the library's stream still uses it, even when the owning Python object
is dropped at once (the caching allocator must not give it to a tensor on
another stream until that work has finished)."""
from __future__ import annotations

import pytest

import tsp_inputs
from gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_colony_workspace_outlives_queued_work():
    import torch
    from paper_1101_2678_amd.aco import Colony

    side = torch.cuda.Stream()
    _, d = tsp_inputs.instance(2400, "uniform", side=1_000_000, seed=1)
    col = Colony(d, 2400, 1, 2, 0.5, 1, atomic=False, stream=side)
    col.attach_nn(30)
    nbytes = col.workspace.numel()
    side.synchronize()
    log("  queue three constructions on a side stream, then drop the context")
    for it in range(3):
        col.construct(it)        # each writes tours, successor tables, lengths
    col.construct_nn(3)
    col.close()
    del col
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    x.fill_(7)
    torch.cuda.synchronize()
    assert bool((x == 7).all()), "a dropped context's workspace was reused while its kernels ran"


def test_batch_workspace_outlives_queued_work():
    import torch
    from paper_1101_2678_amd.aco import Batch

    dists, params = [], []
    for q, n in enumerate([2000, 1500, 1000]):
        dists.append(tsp_inputs.instance(n, "uniform", side=1_000_000, seed=q + 1)[1])
        params.append(dict(m=n, seed=q + 1))
    b = Batch(dists, params)
    b.sync()
    nbytes = b.workspace.numel()
    b.run(3, graph=False)
    b.close()
    del b
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    x.fill_(9)
    torch.cuda.synchronize()
    assert bool((x == 9).all()), "a dropped batch's workspace was reused while its kernels ran"
