"""Host logic of bench.py that runs without a GPU: the algorithmic byte
models, the whole-job roofline record, the oracle timing record and the
refusal of more than one GPU."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

import tsp_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b

    return b


def test_construct_bytes_hand_count(bench):
    # every ant-step reads the current city's n-entry binary32 row: m (n - 1) steps
    assert bench.construct_bytes(3, 2) == 2 * 2 * 4 * 3
    assert bench.construct_bytes(2400, 2400) == 55_272_960_000


def test_update_byte_models_hand_count(bench):
    n, m = 10, 4
    # gather: tau r/w, dist r, choice w (16 n^2), succ/pred rows (4 m n), deposits (4 m)
    assert bench.gather_bytes(n, m) == 16 * 100 + 4 * 40 + 16
    # direct atomic: tours (2 m (n + 1)), deposits (4 m), m n atomics of 16 B, epilogue 24 n^2
    assert bench.atomic_bytes(n, m) == 2 * 4 * 11 + 16 + 16 * 40 + 24 * 100
    # shared-memory atomic: successor table (2 m n), deposits (4 m), epilogue 24 n^2
    assert bench.atomic_shared_bytes(n, m) == 2 * 40 + 16 + 24 * 100


def test_job_roofline_record(bench):
    rec = bench.job_roofline(8e12, 2.0, 100)
    assert rec["bound"] == "hbm" and rec["unit"] == "GB/s" and rec["peak"] == 8000.0
    assert rec["achieved"] == 4000.0 and rec["frac"] == 0.5
    # reading 8 TB at 8 TB/s takes one second: 100 solves per second at the bound
    assert rec["hbm_bound_solves_per_s"] == 100.0
    assert rec["traffic"] is None and rec["algorithmic_bytes"] == 8_000_000_000_000


def test_cpu_baseline_record(bench):
    _, d = tsp_inputs.instance(60, "uniform", side=10_000, seed=3)
    rec = bench.cpu_baseline(d, 60, 0.5)
    assert rec["kind"] == "oracle" and rec["unit"] == "ant-steps/s"
    assert 1 <= rec["cores"] <= 16
    assert rec["value"] > 0 and rec["one_core_construct_ant_steps_per_s"] > 0
    assert rec["sample"] and rec["cpu_model"]


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, cwd=ROOT)
    assert out.returncode == 2
    rec = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in rec["error"]


def test_requested_bytes_hand_count(bench):
    import numpy as np

    # n = 8, tour 0..7: group {0..3} is last needed at step 3, group {4..7}
    # at step 7, so the skip path loads 3 + 7 sixteen-byte groups
    t = np.array([[0, 1, 2, 3, 4, 5, 6, 7, 0]], np.uint16)
    assert bench.requested_bytes(t, 8, skip=True) == 16 * (3 + 7)
    assert bench.requested_bytes(t, 8, skip=False) == 16 * 2 * 7
    # n = 6 (groups {0..3}, {4, 5}): tour 5 0 4 1 2 3 -> last positions 5 and 2
    t = np.array([[5, 0, 4, 1, 2, 3, 5]], np.uint16)
    assert bench.requested_bytes(t, 6, skip=True) == 16 * (5 + 2)


def test_kernel_hash_ignores_comments_only(bench):
    """The traffic record's hash changes with the kernel's code, not with a
    comment or the layout of its text."""
    a = "int f(int x) {  // doubles\n    return 2 * x; /* twice */ }\n"
    b = "int f(int x) {\n  return 2 * x;\n}  // twice x\n"
    c = "int f(int x) { return 3 * x; }"
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)
    assert "doubles" not in bench.code_text(a) and "twice" not in bench.code_text(a)
