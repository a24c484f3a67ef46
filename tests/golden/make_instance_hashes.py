"""Writes instance_hashes.json: SHA-256 fingerprints of the coordinates of the
seeded workloads, so that a change of the generator (or of numpy's random
streams) cannot silently change what the tests and the benchmark run on.
Calls only tsp_inputs.  Run from the repository root:
    python tests/golden/make_instance_hashes.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tsp_inputs  # noqa: E402

WORKLOADS = [  # (n, layout, side, seed): the benchmark and test configurations
    (100, "uniform", 10_000, 1),
    (1000, "uniform", 1_000_000, 1),
    (1000, "cluster", 1_000_000, 1),
    (2400, "uniform", 1_000_000, 1),
    (2400, "cluster", 1_000_000, 1),
    (4096, "uniform", 1_000_000, 4096),
]


def fingerprint(n, layout, side, seed) -> str:
    xy, _ = tsp_inputs.instance(n, layout, side=side, seed=seed)
    return hashlib.sha256(xy.astype("<i8").tobytes()).hexdigest()


if __name__ == "__main__":
    out = {f"{n}-{layout}-{side}-{seed}": fingerprint(n, layout, side, seed)
           for n, layout, side, seed in WORKLOADS}
    with open(os.path.join(HERE, "instance_hashes.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
