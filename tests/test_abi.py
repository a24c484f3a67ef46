"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/aco.h, and rejects invalid arguments before touching the
device."""
from __future__ import annotations

import ast
import ctypes
import os
import re

import numpy as np
import pytest

import tsp_inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aco.h")


@pytest.fixture(scope="module")
def aco():
    from paper_1101_2678_amd import aco as mod

    return mod


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aco_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ["aco_init", "aco_construct", "aco_update", "aco_solve", "aco_workspace_bytes",
                 "aco_read_tours", "aco_read_tau", "aco_destroy", "aco_status_str"]:
        assert must in names


def test_library_exports_every_declared_symbol(aco):
    missing = [f for f in declared_functions() if not hasattr(aco.lib, f)]
    assert not missing, missing


def test_status_strings(aco):
    for s in range(5):
        assert aco.lib.aco_status_str(s)
    assert aco.lib.aco_status_str(99) == b"unknown status"


def test_workspace_bytes(aco):
    P = aco.Params
    ok = P(2400, 2400, 1, 2, 0.5, 1)
    base = aco.lib.aco_workspace_bytes(ctypes.byref(ok), 0)
    full = aco.lib.aco_workspace_bytes(ctypes.byref(ok), 1)
    ld = 2432
    assert full - base >= 8 * 2400 * ld  # the binary64 deposit matrix
    assert base >= 12 * 2400 * ld + 2 * 2400 * 2432 + 4 * 2400 * 2432
    assert base % 256 == 0 and full % 256 == 0
    for bad in [P(2, 5, 1, 2, 0.5, 1), P(4097, 5, 1, 2, 0.5, 1), P(10, 0, 1, 2, 0.5, 1),
                P(10, 65536, 1, 2, 0.5, 1), P(10, 5, 3, 2, 0.5, 1), P(10, 5, 1, 5, 0.5, 1),
                P(10, 5, 1, -1, 0.5, 1), P(10, 5, 1, 2, 0.0, 1), P(10, 5, 1, 2, 1.5, 1),
                P(10, 5, 1, 2, float("nan"), 1)]:
        assert aco.lib.aco_workspace_bytes(ctypes.byref(bad), 1) == 0


def _init(aco, params, dist, ws=0x100000, nbytes=1 << 40):
    ctx = ctypes.c_void_p()
    d = np.ascontiguousarray(dist, np.int32)
    st = aco.lib.aco_init(ctypes.byref(ctx), ctypes.byref(params),
                          d.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ws), nbytes, None)
    return st, ctx


def test_init_rejects_invalid_input_before_device(aco):
    """Every rejection below happens on the host, before any HIP call."""
    _, d = tsp_inputs.instance(10, "uniform", side=1000, seed=1)
    P = aco.Params
    st, ctx = _init(aco, P(10, 5, 1, 2, 0.0, 1), d)
    assert st == aco.ACO_ERR_INVALID and not ctx.value
    asym = d.copy()
    asym[0, 1] += 1
    assert _init(aco, P(10, 5, 1, 2, 0.5, 1), asym)[0] == aco.ACO_ERR_INVALID
    assert b"symmetric" in aco.lib.aco_last_error()
    diag = d.copy()
    diag[3, 3] = 1
    assert _init(aco, P(10, 5, 1, 2, 0.5, 1), diag)[0] == aco.ACO_ERR_INVALID
    zero = d.copy()
    zero[2, 5] = zero[5, 2] = 0
    assert _init(aco, P(10, 5, 1, 2, 0.5, 1), zero)[0] == aco.ACO_ERR_INVALID
    # distances spanning too many binades for exact binary64 deposit sums
    # (a ring of unit edges with chords of 2^30: tours from 10 to 10 * 2^30)
    wild = np.full((10, 10), 2**30, np.int32)
    for i in range(10):
        wild[i, (i + 1) % 10] = wild[(i + 1) % 10, i] = 1
    np.fill_diagonal(wild, 0)
    assert _init(aco, P(10, 65535, 1, 2, 0.5, 1), wild)[0] == aco.ACO_ERR_INVALID
    # workspace: misaligned, too small, NULL
    assert _init(aco, P(10, 5, 1, 2, 0.5, 1), d, ws=0x100010)[0] == aco.ACO_ERR_NOMEM
    assert _init(aco, P(10, 5, 1, 2, 0.5, 1), d, nbytes=1000)[0] == aco.ACO_ERR_NOMEM
    assert _init(aco, P(10, 5, 1, 2, 0.5, 1), d, ws=0)[0] == aco.ACO_ERR_NOMEM
    # NULL arguments
    assert aco.lib.aco_init(None, None, None, None, 0, None) == aco.ACO_ERR_INVALID


def test_calls_on_null_context(aco):
    assert aco.lib.aco_construct(None, 0) == aco.ACO_ERR_INVALID
    assert aco.lib.aco_update(None, 0) == aco.ACO_ERR_INVALID
    assert aco.lib.aco_solve(None, 1, 0, None, None) == aco.ACO_ERR_INVALID
    assert aco.lib.aco_sync(None) == aco.ACO_ERR_INVALID
    aco.lib.aco_destroy(None)


def test_probe_and_select_validation(aco):
    sel = aco.lib.aco_test_select
    assert sel(8, 0, 1, 16, 16, 16, 16, None) == aco.ACO_ERR_INVALID
    assert sel(8, 4097, 1, 16, 16, 16, 16, None) == aco.ACO_ERR_INVALID
    assert sel(8, 10, -1, 16, 16, 16, 16, None) == aco.ACO_ERR_INVALID
    assert sel(8, 10, 1, None, 16, 16, 16, None) == aco.ACO_ERR_INVALID
    assert sel(4, 1025, 1, 16, 16, 16, 16, None) == aco.ACO_ERR_INVALID  # tile 4: n <= 1024
    assert sel(6, 100, 1, 16, 16, 16, 16, None) == aco.ACO_ERR_INVALID
    assert sel(8, 10, 0, None, None, None, None, None) == aco.ACO_OK
    assert aco.lib.aco_probe_copy(16, 16, 15, None) == aco.ACO_ERR_INVALID
    assert aco.lib.aco_probe_read(16, 32, -1, 16, None) == aco.ACO_ERR_INVALID
    rows = aco.lib.aco_probe_rows
    assert rows(16, 0, 64, 64, 1, 1, 16, None) == aco.ACO_ERR_INVALID
    assert rows(16, 10, 60, 64, 1, 1, 16, None) == aco.ACO_ERR_INVALID  # ld < row_len
    assert rows(16, 10, 66, 64, 1, 1, 16, None) == aco.ACO_ERR_INVALID  # ld % 4
    assert rows(16, 10, 4160, 4097, 1, 1, 16, None) == aco.ACO_ERR_INVALID


def test_tile_table(aco):
    aco.reset_tiles()
    # default: tile 4 up to n = 256, 8 above
    assert [aco.get_tile(n) for n in (3, 256, 257, 2400, 4096)] == [4, 4, 8, 8, 8]
    with pytest.raises(aco.AcoError):
        aco.set_tile(900, 1100, 4)  # tile 4 stops at n = 1024
    with pytest.raises(aco.AcoError):
        aco.set_tile(10, 5, 8)
    with pytest.raises(aco.AcoError):
        aco.set_tile(10, 20, 5)
    aco.set_tile(1, 4096, 8)
    aco.set_tile(100, 200, 4)
    assert [aco.get_tile(n) for n in (99, 100, 200, 201)] == [8, 4, 4, 8]
    aco.reset_tiles()
    assert [aco.get_tile(n) for n in (150, 300)] == [4, 8]


def test_shape_table(aco):
    """Several wavefronts per ant: n <= 1024, at least as many passes of
    64 * tile cities as waves; tile 8 with 2 waves, tile 4 with 2, or with 4
    at four passes.  Rejected ranges leave the table unchanged."""
    aco.reset_tiles()
    assert [aco.get_waves(n) for n in (3, 1000, 4096)] == [1, 1, 1]
    aco.set_shape(513, 1024, 8, 2)
    aco.set_shape(257, 512, 4, 2)
    aco.set_shape(769, 1024, 4, 4)
    assert [(aco.get_tile(n), aco.get_waves(n)) for n in (256, 257, 512, 513, 768, 769, 1024,
                                                         1025)] == [
        (4, 1), (4, 2), (4, 2), (8, 2), (8, 2), (4, 4), (4, 4), (8, 1)]
    for bad in ((512, 600, 8, 2),    # n = 512 is one pass of tile 8
                (200, 300, 4, 2),    # n <= 256 is one pass of tile 4
                (700, 800, 4, 4),    # three passes below 769
                (1000, 1100, 8, 2),  # beyond 1024 cities
                (600, 700, 8, 4), (600, 700, 4, 3), (600, 700, 4, 8)):
        with pytest.raises(aco.AcoError):
            aco.set_shape(*bad)
    assert aco.get_waves(1000) == 4 and aco.get_waves(600) == 2
    aco.set_tile(1, 1024, 8)  # the tile setter means one wavefront
    assert aco.get_waves(1000) == 1
    aco.reset_tiles()
    assert [(aco.get_tile(n), aco.get_waves(n)) for n in (100, 1000)] == [(4, 1), (8, 1)]
    sel = aco.lib.aco_test_select_shape
    assert sel(8, 2, 512, 0, None, None, None, None, None) == aco.ACO_ERR_INVALID
    assert sel(4, 4, 700, 0, None, None, None, None, None) == aco.ACO_ERR_INVALID
    assert sel(8, 2, 1000, 1, None, None, None, None, None) == aco.ACO_ERR_INVALID
    assert sel(8, 2, 1000, 0, None, None, None, None, None) == aco.ACO_OK


def test_batch_workspace_and_validation(aco):
    P = aco.Params
    arr = (P * 3)(P(100, 100, 1, 2, 0.5, 1), P(50, 20, 1, 2, 0.5, 2), P(700, 700, 1, 2, 0.5, 3))
    total = aco.lib.aco_batch_workspace_bytes(3, arr)
    single = sum(aco.lib.aco_workspace_bytes(ctypes.byref(arr[q]), 0) for q in range(3))
    assert total >= single + 4 * (100 + 20 + 700) + 4 * (100 + 50 + 700)
    bad = (P * 2)(P(100, 100, 1, 2, 0.5, 1), P(2, 20, 1, 2, 0.5, 2))
    assert aco.lib.aco_batch_workspace_bytes(2, bad) == 0
    assert aco.lib.aco_batch_workspace_bytes(0, arr) == 0
    b = ctypes.c_void_p()
    _, d = tsp_inputs.instance(10, "uniform", side=1000, seed=1)
    asym = d.copy()
    asym[1, 2] += 1
    one = (P * 1)(P(10, 5, 1, 2, 0.5, 1))
    ptrs = (ctypes.c_void_p * 1)(asym.ctypes.data)
    assert aco.lib.aco_batch_init(ctypes.byref(b), 1, one, ptrs, 0x100000, 1 << 40,
                                  None) == aco.ACO_ERR_INVALID
    assert b"instance 0" in aco.lib.aco_last_error()
    assert aco.lib.aco_batch_run(None, 1, 0) == aco.ACO_ERR_INVALID
    aco.lib.aco_batch_destroy(None)


def test_autotune_validation(aco):
    sizes = (ctypes.c_int32 * 2)(200, 100)
    assert aco.lib.aco_autotune(0x100000, 1 << 40, sizes, 2, 1, None, None, None,
                                None) == aco.ACO_ERR_INVALID  # not increasing
    sizes = (ctypes.c_int32 * 1)(2)
    assert aco.lib.aco_autotune(0x100000, 1 << 40, sizes, 1, 1, None, None, None,
                                None) == aco.ACO_ERR_INVALID
    sizes = (ctypes.c_int32 * 1)(100)
    assert aco.lib.aco_autotune(0x100000, 10, sizes, 1, 1, None, None, None,
                                None) == aco.ACO_ERR_NOMEM


def test_server_validation(aco):
    assert aco.lib.aco_server_table_bytes(0, 10, 10, 1) == 0
    assert aco.lib.aco_server_table_bytes(10, 0, 10, 1) == 0
    assert aco.lib.aco_server_table_bytes(10, 10, 10, 9) == 0
    head = aco.lib.aco_server_table_bytes(4, 100, 100, 1)
    assert head >= 4 * 64 + 400 + 400 and head % 256 == 0
    assert aco.lib.aco_server_table_bytes(4, 100, 100, 3) == 3 * head
    s = ctypes.c_void_p()
    b1 = (ctypes.c_int32 * 1)(4096)
    b2 = (ctypes.c_int32 * 2)(500, 400)
    assert aco.lib.aco_server_create(ctypes.byref(s), None, 1 << 20, 4, 100, 100, 1,
                                     b1) == aco.ACO_ERR_NOMEM
    assert aco.lib.aco_server_create(ctypes.byref(s), 0x100000, 16, 4, 100, 100, 1,
                                     b1) == aco.ACO_ERR_NOMEM
    assert aco.lib.aco_server_create(ctypes.byref(s), 0x100000, 1 << 20, 0, 100, 100, 1,
                                     b1) == aco.ACO_ERR_INVALID
    assert aco.lib.aco_server_create(ctypes.byref(s), 0x100000, 1 << 20, 4, 100, 100, 2,
                                     b2) == aco.ACO_ERR_INVALID  # bounds not increasing
    assert aco.lib.aco_server_step(None, None) == aco.ACO_ERR_INVALID
    aco.lib.aco_server_destroy(None)


def test_nn_workspace_and_validation(aco):
    """Candidate-list tables: two 256-byte aligned arrays of n x kp entries
    (kp = nn rounded up to 32), uint16 lists and uint64 packed candidates."""
    f = aco.lib.aco_nn_workspace_bytes
    r256 = lambda v: (v + 255) // 256 * 256
    for n, nn in [(3, 1), (3, 2), (100, 30), (2400, 30), (4096, 64), (65, 33)]:
        kp = (nn + 31) // 32 * 32
        assert f(n, nn) == r256(n * kp * 2) + r256(n * kp * 8), (n, nn)
    for n, nn in [(3, 3), (3, 0), (100, 65), (2, 1), (4097, 30), (100, -1)]:
        assert f(n, nn) == 0, (n, nn)
    # calls on a NULL context fail cleanly, before any device work
    for fn, args in [(aco.lib.aco_nn_attach, (None, 30, None, 0)),
                     (aco.lib.aco_construct_nn, (None, 0)),
                     (aco.lib.aco_solve_nn, (None, 1, 0, None, None)),
                     (aco.lib.aco_read_nn_lists, (None, None))]:
        assert fn(*args) == aco.ACO_ERR_INVALID


def test_product_entry_points_validate(aco):
    """Product rule and Philox probe: bad arguments fail before device work."""
    L = aco.lib
    assert L.aco_construct_product(None, 0) == aco.ACO_ERR_INVALID
    assert L.aco_solve_product(None, 1, 0, None, None) == aco.ACO_ERR_INVALID
    sel = L.aco_test_product_select
    assert sel(0, 1, 16, 16, 16, 16, None) == aco.ACO_ERR_INVALID        # n < 1
    assert sel(4097, 1, 16, 16, 16, 16, None) == aco.ACO_ERR_INVALID     # n > 4096
    assert sel(10, -1, 16, 16, 16, 16, None) == aco.ACO_ERR_INVALID      # count < 0
    assert sel(10, 1, None, 16, 16, 16, None) == aco.ACO_ERR_INVALID     # NULL rows
    assert sel(10, 1, 8, 16, 16, 16, None) == aco.ACO_ERR_INVALID        # misaligned rows
    assert sel(10, 0, None, None, None, None, None) == aco.ACO_OK        # nothing to do
    assert L.aco_probe_philox(-1, 1, 0, None, None) == aco.ACO_ERR_INVALID
    assert L.aco_probe_philox(1, 1, 0, None, None) == aco.ACO_ERR_INVALID
    assert L.aco_probe_philox(0, 1, 0, None, None) == aco.ACO_OK


def test_binding_loads_torch_hip_runtime():
    """Importing the binding before torch must not bring a second HIP runtime
    into the process: exactly one libamdhip64 is mapped, torch's."""
    import subprocess
    import sys

    code = ("from paper_1101_2678_amd import aco\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(sorted({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         check=True).stdout
    libs = ast.literal_eval(out.strip().splitlines()[-1])
    assert len(libs) == 1 and os.sep + "torch" + os.sep in libs[0], libs



def test_distance_input_is_checked_not_cast(aco):
    """Distances reach the library unchanged: integer input is converted to
    int32 only when it fits, anything else is refused."""
    ok = aco.as_dist(np.array([[0, 7], [7, 0]], np.int64))
    assert ok.dtype == np.int32 and ok.flags["C_CONTIGUOUS"] and ok[0, 1] == 7
    with pytest.raises(TypeError):
        aco.as_dist(np.array([[0.0, 1.5], [1.5, 0.0]]))
    with pytest.raises(ValueError):
        aco.as_dist(np.array([[0, 2**40], [2**40, 0]], np.int64))
    with pytest.raises(ValueError):
        aco.as_dist(np.zeros((2, 3), np.int32))
