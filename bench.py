#!/usr/bin/env python3
"""Benchmark of the Ant System hot path on one MI355X.

A step is one AS iteration over the resident instance: tour construction by
all m ants (Section II, Eq. 1), then the best-so-far tour and the pheromone
update (Eqs. 2-4, gather variant) with the choice refresh.  The headline
workload is n = m = 2400 cities uniform in [0, 10^6]^2 (the largest size the
paper measures), alpha = 1, beta = 2, rho = 0.5, Philox seed 1; the instance
and all state are resident in HBM before timing starts.

Prints one JSON line.  `value` is ant-steps per second of the whole step
(m (n-1) roulette selections per step).  The construction roofline is taken
against the streaming read bandwidth measured live at the choice matrix's
own footprint (the Infinity Cache at n = 2400), with the published HBM peak
beside it; each update kernel is set against one copy launch over its own
footprint.  Further fields: per-kernel times from HIP events on the launch
stream, the counter traffic when it was taken on the current kernel source,
HBM and 160 MB streaming probes, the same steps with candidate-list
construction (`nn_list`) and with the product-and-argmax rule (`product`),
the oracle timed on a bounded sample on the host (`cpu_baseline`), and under
`configs` every other workload: n = 100, n = 1000 (uniform and 20-cluster),
256 uneven instances as one graph-replayed batch against one instance per
launch (`batch256`, solves/s), and a Poisson trace through the
continuous-batching server against one request at a time (`served`, solves/s
with p50 and p99).

`--workload NAME` runs one of them alone.  Profiled runs add
`--sync-launches`.  The library runs on one GPU: `--gpus` other than 1 exits
with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import tsp_inputs  # noqa: E402

METRIC = ("construction ant-steps/s + update GB/s (% roofline); served solves/s and p99")
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published

WORKLOADS = {
    "n2400": dict(n=2400, m=2400, layout="uniform", side=1_000_000, seed=1),
    "n1000u": dict(n=1000, m=1000, layout="uniform", side=1_000_000, seed=1),
    "n1000c": dict(n=1000, m=1000, layout="cluster", side=1_000_000, seed=1),
    "n100": dict(n=100, m=100, layout="uniform", side=10_000, seed=1),
}
ALPHA, BETA, RHO = 1, 2, 0.5
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "construct_n2400_traffic.json")
# The text the construction kernel is compiled from: its source, the headers
# of its device code, and (of the state header, which also declares host
# launchers) the colony struct it takes as its argument.
KERNEL_SOURCES = ["paper_1101_2678_amd/csrc/construct.hip", "paper_1101_2678_amd/csrc/r64_lanes.hpp",
                  "paper_1101_2678_amd/csrc/aco_device.hpp"]
KERNEL_STRUCT = ("paper_1101_2678_amd/csrc/aco_state.hpp", "struct Colony {", "};")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def code_text(text: str) -> str:
    """Source text without its comments, whitespace runs collapsed: what
    the compiler sees, so that editing a comment does not mark the kernel as
    changed."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(code_text(f.read()).encode())
    rel, start, end = KERNEL_STRUCT
    with open(os.path.join(ROOT, rel)) as f:
        text = f.read()
    i = text.index(start)
    h.update(code_text(text[i:text.index(end, i) + len(end)]).encode())
    return h.hexdigest()


def construct_bytes(n: int, m: int) -> int:
    """Algorithmic bytes of one construction launch: every ant-step streams
    the n-entry binary32 choice row of its current city."""
    return 4 * n * m * (n - 1)


def job_roofline(con_bytes: float, seconds: float, solves: int) -> dict:
    """Whole-job bandwidth of a many-instance workload: the choice-row bytes
    every construction of every solve must read (4 n m (n - 1) per iteration),
    over the wall time of the job (updates, best-so-far and gaps included);
    with the solves/s that reading them at the HBM peak alone would allow."""
    achieved = con_bytes / seconds / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
            "scope": "whole job: construction bytes of every solve / wall time",
            "algorithmic_bytes": int(con_bytes),
            "hbm_bound_solves_per_s": round(solves / (con_bytes / (HBM_PEAK_GBPS * 1e9)), 3)}


def gather_bytes(n: int, m: int) -> int:
    """tau read+write, distances read, choice write (16 n^2), the succ/pred
    neighbour tables (4 m n) and the deposits (4 m)."""
    return 16 * n * n + 4 * m * n + 4 * m


def atomic_bytes(n: int, m: int) -> int:
    """Direct atomic update: tours (2 m (n+1)) and deposits (4 m) read, m n
    binary64 atomics into the upper triangle (8 B read + 8 B write each);
    epilogue: tau r/w, dist r, choice w (16 n^2) and the upper-triangle
    deposits read and cleared (8 n^2)."""
    return 2 * m * (n + 1) + 4 * m + m * n * 16 + 24 * n * n


def atomic_shared_bytes(n: int, m: int) -> int:
    """Atomic update with the deposits combined in shared memory: the
    successor table (2 m n) and the deposits (4 m) read, then the epilogue of
    the direct variant (24 n^2).  The global atomics, one per distinct edge
    of a row's workgroup, depend on the tours and are not counted."""
    return 2 * m * n + 4 * m + 24 * n * n


UPDATE_BYTES = {"gather": gather_bytes, "atomic": atomic_shared_bytes,
                "atomic_direct": atomic_bytes}


def traffic_from_profile():
    """HBM bytes per construction launch measured by rocprofv3 counters
    (FETCH_SIZE + WRITE_SIZE, calibrated on a copy kernel), if they were taken
    on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None, "no counter record"
    if rec.get("source_sha256") != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    return int(rec["bytes_per_launch"]), rec.get("note", "")


def cpu_baseline(d: np.ndarray, m: int, seconds: float):
    """The oracle as it stands on the host's cores (up to 16 threads, the
    host share of one GPU): ants of iteration 0, each one serial oracle call,
    built by a pool of threads until `seconds` pass, then one update (a
    serial oracle call) with m tours made by tiling those ants (the update's
    cost does not depend on which tours)."""
    import itertools
    import threading
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    n = d.shape[0]
    st = oracle.init(d, m, ALPHA, BETA, RHO, 1)
    threads = max(1, min(16, os.cpu_count() or 1))
    tours, lens = [], []
    lock = threading.Lock()
    counter = itertools.count()
    t0 = time.perf_counter()
    deadline = t0 + seconds

    def worker():
        while time.perf_counter() < deadline:
            k = next(counter)
            if k >= m:
                return
            t, ln = oracle.construct_ant(st.choice, d, 1, 0, k)   # ctypes drops the GIL
            with lock:
                tours.append(t)
                lens.append(ln)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        for f in [ex.submit(worker) for _ in range(threads)]:
            f.result()
    t_construct = time.perf_counter() - t0
    k = len(tours)
    reps = (m + k - 1) // k
    all_t = np.tile(np.array(tours), (reps, 1))[:m]
    all_l = np.tile(np.array(lens, np.int64), reps)[:m]
    t1 = time.perf_counter()
    oracle.update(st.tau, all_t, all_l, d, RHO, ALPHA, BETA)
    t_update = time.perf_counter() - t1
    per_ant = t_construct / k
    step_s = per_ant * m + t_update
    # one host core: the same serial calls, one after another, for a quarter
    # of the budget (at least one ant)
    t2 = time.perf_counter()
    solo = 0
    while solo == 0 or (time.perf_counter() - t2 < seconds / 4 and solo < m):
        oracle.construct_ant(st.choice, d, 1, 0, solo)
        solo += 1
    t_solo = time.perf_counter() - t2
    return {
        "value": m * (n - 1) / step_s,
        "unit": "ant-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{k} ants of iteration 0 at n={n} ({k * (n - 1)} ant-steps) built by "
                   f"{threads} threads in {t_construct:.1f} s, plus one full update with m={m} "
                   f"tours ({t_update:.2f} s, one thread); step time extrapolated to m={m} ants"),
        "construct_ant_steps_per_s": (n - 1) / per_ant,
        "update_s": t_update,
        "step_s_extrapolated": step_s,
        "one_core_construct_ant_steps_per_s": solo * (n - 1) / t_solo,
        "one_core_sample": f"{solo} ants of iteration 0 built one after another in {t_solo:.1f} s",
        "cpu_model": host_cpu_model(),
    }


def host_cpu_model() -> str:
    """The host processor's model name and logical CPU count, as the kernel reports them."""
    try:
        with open("/proc/cpuinfo") as f:
            names = [ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")]
    except OSError:
        return "unknown"
    return f"{names[0]} ({len(names)} logical CPUs)" if names else "unknown"


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


PROBE_SHAPES = ((4, False), (16, False), (8, True))  # (loads in flight, nontemporal)


def stream_read_ceiling(torch, aco, nbytes: int, min_ms: float = 5.0) -> dict:
    """Streaming read bandwidth of a buffer of `nbytes` (aco_probe_read_shape:
    each of the eight XCDs walks the whole buffer, so every XCD's L2 sees the
    full footprint, as in tour construction), the best over PROBE_SHAPES,
    each timed with HIP events on the launch stream over at least `min_ms`.
    A footprint above the 4 MB L2 of an XCD and within the 256 MB Infinity
    Cache measures the Infinity Cache (MALL); one well above 256 MB measures
    HBM."""
    stream = torch.cuda.current_stream()
    buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    sink = torch.zeros(4096, dtype=torch.float32, device="cuda")
    best, shapes = None, {}
    for loads, nt in PROBE_SHAPES:
        aco.probe_read(buf, 8, sink, loads=loads, nontemporal=nt)  # every XCD touches it once
        reps, ms = 8, 0.0
        for _ in range(12):
            e0, e1 = _events(torch)
            e0.record(stream)
            aco.probe_read(buf, reps, sink, loads=loads, nontemporal=nt)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            if ms >= min_ms:
                break
            reps = int(reps * min(64.0, max(2.0, 1.3 * min_ms / max(ms, 1e-3))) + 7) // 8 * 8
        rate = nbytes * reps / (ms * 1e-3) / 1e9
        shapes[f"{loads}{'nt' if nt else ''}"] = round(rate, 1)
        if best is None or rate > best["GBps"]:
            best = {"GBps": round(rate, 1), "bytes": int(nbytes), "reps": reps, "ms": round(ms, 3),
                    "loads_in_flight": loads, "nontemporal": nt}
    del buf
    best["by_shape_GBps"] = shapes
    return best


def copy_ceiling(torch, aco, nbytes: int, launches: int = 20) -> dict:
    """Read-plus-write bandwidth of one aco_probe_copy launch over a footprint
    of `nbytes` (half source, half destination), the mean of `launches`
    single launches each timed with HIP events: the same footprint and the
    same launch granularity as one update kernel."""
    stream = torch.cuda.current_stream()
    half = (nbytes // 2) // 16 * 16
    src = torch.ones(half // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    aco.probe_copy(dst, src)
    times = []
    for _ in range(launches):
        e0, e1 = _events(torch)
        e0.record(stream)
        aco.probe_copy(dst, src)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del src, dst
    ms = float(np.mean(times))
    return {"GBps": round(2 * half / (ms * 1e-3) / 1e9, 1), "bytes": 2 * half,
            "ms_per_launch": round(ms, 4)}


def random_rows_rate(torch, aco, n: int, m: int, rows: int) -> float:
    """GB/s of aco_probe_rows: m one-wave workgroups each read n - 1 random
    whole rows of n floats from a rows x ld matrix (the construction's access
    pattern without its arithmetic)."""
    stream = torch.cuda.current_stream()
    ld = (n + 63) // 64 * 64
    sink = torch.zeros(max(m, 4096), dtype=torch.float32, device="cuda")
    mat = torch.rand(rows * ld, dtype=torch.float32, device="cuda")
    aco.probe_rows(mat, rows, ld, n, m, 8, sink)
    e0, e1 = _events(torch)
    e0.record(stream)
    aco.probe_rows(mat, rows, ld, n, m, n - 1, sink)
    e1.record(stream)
    torch.cuda.synchronize()
    del mat
    return round(4.0 * n * m * (n - 1) / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)


def random_rows_ceiling(torch, aco, n: int, m: int, waves_factors=(1, 2, 4, 8),
                        in_flight=(1, 2)) -> dict:
    """Best rate of reading random whole rows of an n x ld matrix (the choice
    matrix's footprint) with 1, 2, 4 and 8 times m one-wave workgroups, each
    keeping one or two rows in flight: the memory system's limit for this
    access pattern, where each XCD's L2 keeps a share of the rows (a
    sequential sweep of the footprint keeps none), measured with up to
    sixteen times the rows construction has in flight."""
    stream = torch.cuda.current_stream()
    ld = (n + 63) // 64 * 64
    sink = torch.zeros(max(8 * m, 4096), dtype=torch.float32, device="cuda")
    mat = torch.rand(n * ld, dtype=torch.float32, device="cuda")
    by = {}
    for f in waves_factors:
        for r in in_flight:
            waves = f * m
            steps = max(16, m * (n - 1) // (2 * waves))
            steps += (-steps) % r
            aco.probe_rows(mat, n, ld, n, waves, 4, sink, rows_in_flight=r)
            e0, e1 = _events(torch)
            e0.record(stream)
            aco.probe_rows(mat, n, ld, n, waves, steps, sink, rows_in_flight=r)
            e1.record(stream)
            torch.cuda.synchronize()
            by[f"{waves}x{r}"] = round(4.0 * n * waves * steps / (e0.elapsed_time(e1) * 1e-3) / 1e9,
                                       1)
    del mat
    best = max(by, key=by.get)
    return {"GBps": by[best], "shape": best, "by_shape_GBps": by}


def requested_bytes(tours: np.ndarray, n: int, skip: bool) -> int:
    """Bytes the construction kernel asks the memory system for in one launch
    (16-byte loads of 4-city groups).  With the skip path a group is loaded
    at step s only if one of its cities is still unvisited, i.e. at steps
    1 .. (last position of the group's cities in the tour); without it every
    group of the row is loaded at all n - 1 steps."""
    groups = (n + 3) // 4
    m = tours.shape[0]
    if not skip:
        return 16 * groups * (n - 1) * m
    total = 0
    for k0 in range(0, m, 256):
        t = tours[k0:k0 + 256, :n].astype(np.int64)
        pos = np.full((t.shape[0], groups * 4), -1, np.int64)
        np.put_along_axis(pos, t, np.arange(n, dtype=np.int64)[None, :], axis=1)
        total += int(pos.reshape(t.shape[0], groups, 4).max(axis=2).sum())
    return 16 * total


SYNC_LAUNCHES = False


def launched(torch):
    """After a launch: wait for it when --sync-launches is given.  Profiled
    runs use it: under rocprofv3 on these GPUs, launches queued back to back
    on one stream did not reliably see each other's results (the host
    synchronising in between restores them), while per-kernel durations are
    the same either way."""
    if SYNC_LAUNCHES:
        torch.cuda.synchronize()


def nn_fallback_steps(tours: np.ndarray, nnl: np.ndarray, chunk: int = 128) -> int:
    """Steps at which every candidate of the current city was already
    visited (the ant then scans the whole choice row)."""
    m, n1 = tours.shape
    n = n1 - 1
    steps = np.arange(1, n, dtype=np.int32)[None, :, None]
    total = 0
    for k0 in range(0, m, chunk):
        t = tours[k0:k0 + chunk].astype(np.int64)
        c = t.shape[0]
        pos = np.empty((c, n), np.int32)                    # step at which a city is visited
        np.put_along_axis(pos, t[:, :-1], np.arange(n, dtype=np.int32)[None, :], axis=1)
        cand = nnl[t[:, :n - 1]].reshape(c, -1).astype(np.int64)  # lists of tour[s-1]
        cpos = np.take_along_axis(pos, cand, axis=1).reshape(c, n - 1, -1)
        total += int((cpos < steps).all(axis=2).sum())
    return total


def nn_lists_problem(d: np.ndarray, nnl: np.ndarray):
    """None if every row lists other cities in non-decreasing distance, else
    what is wrong (a property check, independent of how lists are built)."""
    n = d.shape[0]
    if nnl.max() >= n:
        return f"a list entry is >= n ({int(nnl.max())})"
    if (nnl == np.arange(n)[:, None]).any():
        return "a row lists its own city"
    dd = np.take_along_axis(d, nnl.astype(np.int64), axis=1)
    if (np.diff(dd, axis=1) < 0).any():
        return "a list is not ordered by distance"
    return None


def bench_nn(torch, aco, d, m: int, nn: int, steps: int, warmup: int, update: str, cpu_s: float):
    """Candidate-list construction (nn nearest cities) on the same instance:
    `steps` iterations timed like the main loop, HIP events around each
    construction (candidate-table refresh included)."""
    n = d.shape[0]
    col = aco.Colony(d, m, ALPHA, BETA, RHO, seed=1, atomic=(update != "gather"))
    col.attach_nn(nn)
    nnl = col.nn_lists()
    problem = nn_lists_problem(d, nnl)
    stream = torch.cuda.current_stream()
    it = 0
    for _ in range(warmup):
        col.construct_nn(it)
        launched(torch)
        col.update(update)
        launched(torch)
        it += 1
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        ev[3 * s].record(stream)
        col.construct_nn(it)
        launched(torch)
        ev[3 * s + 1].record(stream)
        col.update(update)
        launched(torch)
        ev[3 * s + 2].record(stream)
        it += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_con = float(np.mean([ev[3 * s].elapsed_time(ev[3 * s + 1]) for s in range(steps)]))
    tours, _ = col.tours()
    best = col.best()[1]
    col.close()
    if problem is None and not (tours < n).all():
        problem = "a tour holds a city index >= n"
    fb = nn_fallback_steps(tours, nnl) if problem is None else 0
    ant_steps = m * (n - 1)
    frac = fb / ant_steps
    # bytes one construction must move: a packed candidate row (8 B per list
    # entry, padded to 32 entries) per step, a 4n-byte choice row per fallback
    # step, plus the epilogue (d lookups, tours, succ/pred) as in full construction
    kp = (nn + 31) // 32 * 32
    alg = ant_steps * 8 * kp + fb * 4 * n + m * (n * 4 + 2 * (n + 1) + 4 * n)
    out = {
        "nn": nn,
        "ms_per_step": round(wall * 1e3 / steps, 4),
        "value": round(ant_steps / wall * steps, 1),
        "unit": "ant-steps/s",
        "construct_ms": round(t_con, 4),
        "construct_ant_steps_per_s": round(ant_steps / (t_con * 1e-3), 1),
        "fallback_fraction_last_iter": round(frac, 5),
        "construct_algorithmic_bytes": int(alg),
        "construct_GBps": round(alg / (t_con * 1e-3) / 1e9, 1),
        "bound": "latency (one dependent candidate-row load per step)",
        "best_len_after_run": int(best),
    }
    if problem is not None:
        out["error"] = problem
    if cpu_s > 0:
        import oracle

        st = oracle.init(d, m, ALPHA, BETA, RHO, 1)
        lists = oracle.nn_lists(d, nn)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < cpu_s:
            oracle.construct_ant_nn(st.choice, d, lists, 1, 0, k)
            k += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(k * (n - 1) / el, 1), "unit": "ant-steps/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{k} ants of iteration 0 (nn={nn}), one by one"}
    return out


def philox_ceiling(torch, aco, waves_list, steps: int = 200):
    """Philox blocks/s of aco_probe_philox for each wavefront count."""
    out = []
    for waves in waves_list:
        sink = torch.zeros(waves * 64, dtype=torch.int32, device="cuda")
        aco.probe_philox(waves, 5, 1, sink)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        aco.probe_philox(waves, steps, 1, sink)
        e1.record()
        torch.cuda.synchronize()
        out.append(round(waves * 64 * 10 * steps / (e0.elapsed_time(e1) * 1e-3), 1))
    return out


def bench_product(torch, aco, d, m: int, steps: int, warmup: int, update: str, cpu_s: float):
    """The paper's product-and-argmax construction on the same instance:
    `steps` iterations timed like the main loop, HIP events around each
    construction."""
    n = d.shape[0]
    col = aco.Colony(d, m, ALPHA, BETA, RHO, seed=1, atomic=(update != "gather"))
    stream = torch.cuda.current_stream()
    it = 0
    for _ in range(warmup):
        col.construct_product(it)
        launched(torch)
        col.update(update)
        launched(torch)
        it += 1
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        ev[2 * s].record(stream)
        col.construct_product(it)
        launched(torch)
        ev[2 * s + 1].record(stream)
        col.update(update)
        launched(torch)
        it += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_con = float(np.mean([ev[2 * s].elapsed_time(ev[2 * s + 1]) for s in range(steps)]))
    tours, _ = col.tours()
    best = col.best()[1]
    col.close()
    ant_steps = m * (n - 1)
    blocks = ant_steps * ((n + 3) // 4)          # Philox blocks the rule needs
    ceiling = philox_ceiling(torch, aco, [16 * 1024, m])
    out = {
        "ms_per_step": round(wall * 1e3 / steps, 4),
        "value": round(ant_steps / wall * steps, 1),
        "unit": "ant-steps/s",
        "construct_ms": round(t_con, 4),
        "construct_ant_steps_per_s": round(ant_steps / (t_con * 1e-3), 1),
        "philox_blocks_per_launch": int(blocks),
        "philox_blocks_per_s": round(blocks / (t_con * 1e-3), 1),
        "construct_GBps": round(4 * n * ant_steps / (t_con * 1e-3) / 1e9, 1),
        "best_len_after_run": int(best),
        "roofline": {"bound": "alu", "achieved": round(blocks / (t_con * 1e-3), 1),
                     "peak": ceiling[0], "unit": "Philox4x32-10 blocks/s",
                     "frac": round(blocks / (t_con * 1e-3) / ceiling[0], 4),
                     "peak_note": "measured: aco_probe_philox, the same Philox formulation with "
                                  "no loads or selection, 16 wavefronts per SIMD",
                     "ceiling_at_m_wavefronts": ceiling[1],
                     "kernel": "k_construct_product"},
    }
    if not (tours < n).all():
        out["error"] = "a tour holds a city index >= n"
    if cpu_s > 0:
        import oracle

        st = oracle.init(d, m, ALPHA, BETA, RHO, 1)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < cpu_s:
            oracle.construct_ant_product(st.choice, d, 1, 0, k)
            k += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(k * (n - 1) / el, 1), "unit": "ant-steps/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{k} ants of iteration 0, one by one"}
    return out


def bench_batch(args, torch, aco):
    """256 independent instances, n = round(exp(U(ln 50, ln 1000))), m = n,
    uniform cities, alpha 1, beta 2, rho 0.5, 25 iterations each, tiles from
    the autotuner; the batch (one graph replay of 25 iterations x 3 launches)
    against the same set run one instance per launch on one stream."""
    count, iters = 256, 25
    sizes = tsp_inputs.log_uniform_sizes(count, 50, 1000, seed=4)
    dists = [tsp_inputs.instance(int(n), "uniform", side=1_000_000, seed=q + 1)[1]
             for q, n in enumerate(sizes)]
    params = [dict(m=int(n), alpha=ALPHA, beta=BETA, rho=RHO, seed=q + 1)
              for q, n in enumerate(sizes)]
    tune_sizes = [64, 128, 256, 512, 1024]
    tiles, waves, shape_ms = aco.autotune(tune_sizes, reps=3)
    log(f"bench batch: autotune chose tiles {tiles.tolist()} waves {waves.tolist()} "
        f"(ms per shape {aco.SHAPES}: {np.round(shape_ms, 4).tolist()})")
    stream = torch.cuda.Stream()
    b = aco.Batch(dists, params, stream=stream)
    default_cfg = b.config
    # the batched launch's own autotuner: workgroups per CU x tile policy,
    # timed on this batch (each candidate advances it by 3 iterations)
    cands = [(w, t) for t in (-1, 0, 1024) for w in (0, 8, 12, 16, 20, 24, 32)]
    best, cand_ms = b.autotune(cands, iters=2)
    log(f"bench batch: launch autotune chose {cands[best]} ({cand_ms[best]:.3f} ms/iteration; "
        f"default {default_cfg})")
    b.run(iters, graph=True)  # captures the graph and runs 25 iterations
    b.sync()
    t0 = time.perf_counter()
    b.run(iters, graph=True)  # replays it: iterations 25..49
    b.sync()
    t_batch = time.perf_counter() - t0
    # bytes the batched construction asks for (it skips 4-city groups once all
    # are visited), estimated from each instance's last tours
    req_iter = sum(requested_bytes(b.tours(q)[0], int(n), skip=True)
                   for q, n in enumerate(sizes))
    choice_footprint = sum(int(n) * ((int(n) + 63) // 64 * 64) * 4 for n in sizes)
    cols = [aco.Colony(d, p["m"], ALPHA, BETA, RHO, p["seed"], atomic=False, stream=stream)
            for d, p in zip(dists, params)]
    for c in cols:
        for it in range(2):
            c.construct(it)
            c.update("gather")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in cols:
        for it in range(2, 2 + iters):
            c.construct(it)
            c.update("gather")
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    ant_steps = int(sum(int(n) * (int(n) - 1) for n in sizes)) * iters
    rec = {
        "metric": "batched solves/s (25 AS iterations per solve)",
        "value": round(count / t_batch, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(t_batch * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{count} independent instances, n log-uniform in [50, 1000] "
                               f"(sum n = {int(sizes.sum())}), m = n, uniform cities, alpha 1, "
                               f"beta 2, rho 0.5, {iters} iterations each, gather update, "
                               "one HIP graph replay",
                   "count": count, "iterations": iters},
        "one_instance_per_launch": {"seconds": round(t_single, 4),
                                    "solves_per_s": round(count / t_single, 2)},
        "speedup_vs_one_per_launch": round(t_single / t_batch, 2),
        "ant_steps_per_s": round(ant_steps / t_batch, 1),
        "shapes": {"sizes": tune_sizes, "tile": tiles.tolist(), "waves": waves.tolist(),
                   "ms_per_construction": {f"tile{t}_waves{w}": [round(float(x), 4) for x in col]
                                           for (t, w), col in zip(aco.SHAPES, shape_ms.T)},
                   "note": "single-instance construction shape per size (m = n) from the "
                           "autotuner, used by the one-instance-per-launch comparison; the "
                           "batched launch takes only the tile; -1 = shape does not support "
                           "the size"},
        "launch_autotune": {
            "candidates": [{"wg_per_cu": w, "tile4_max_n": t, "ms_per_iteration": round(float(x), 4)}
                           for (w, t), x in zip(cands, cand_ms)],
            "chosen": {"wg_per_cu": cands[best][0], "tile4_max_n": cands[best][1]},
            "default": default_cfg,
            "note": "wg_per_cu: construction workgroups per CU allowed by the LDS request (0 = "
                    "no cap); tile4_max_n: instances up to this n use 4 cities per lane (-1 = "
                    "the tile table above, 0 = all 8)"},
        "roofline": job_roofline(
            float(sum(construct_bytes(int(n), int(n)) for n in sizes)) * iters, t_batch, count),
    }
    rf = rec["roofline"]
    rf["requested_bytes"] = int(req_iter) * iters
    rf["requested_GBps"] = round(req_iter * iters / t_batch / 1e9, 1)
    rf["frac_requested"] = round(rf["requested_GBps"] / HBM_PEAK_GBPS, 4)
    rf["choice_footprint_bytes"] = choice_footprint
    rf["frac_note"] = (
        f"achieved counts every ant-step's whole choice row; the batched kernel asks for "
        f"{req_iter * iters / rf['algorithmic_bytes']:.3f} of those bytes (it skips 4-city groups "
        f"once all are visited; estimated from each instance's last tours), and the "
        f"construction reads only the choice matrices, {choice_footprint / 1e6:.0f} MB "
        f"together, which the Infinity Cache holds and of which the small instances' sit in "
        f"L2, so the whole-job rate can pass the HBM figure")
    aco.reset_tiles()
    return rec


def bench_served(args, torch, aco):
    """Poisson arrivals at 200 requests/s, each asking for 50 AS iterations on
    a fresh instance, n log-uniform in [100, 3000], m = n, uniform or
    20-cluster layout with equal odds, per-request seed; served by the
    continuous batcher (admission by slots and pool memory against free HBM),
    then the same trace served one request at a time on the plain path."""
    import copy

    from paper_1101_2678_amd import serve

    reqs = serve.make_requests(args.requests, 200.0, n_lo=100, n_hi=3000, iters=50, seed=5)
    plain_reqs = copy.deepcopy(reqs)
    free, total = torch.cuda.mem_get_info()
    pool = min(int(free * 0.5), 64 << 30)
    footprint = [r.footprint_bytes() for r in reqs]
    formula = [12 * r.n * r.n + 2 * r.m * r.n for r in reqs]
    fifo_reqs = copy.deepcopy(reqs)
    log(f"bench served: {len(reqs)} requests, pool {pool / 1e9:.1f} GB, slots {args.slots}")
    srv = serve.Server(pool_bytes=pool, max_slots=args.slots)
    batched = serve.run_open_loop(srv, reqs, policy="size")
    srv.close()
    log(f"bench served: batched, size-aware admission {batched}")
    srv = serve.Server(pool_bytes=pool, max_slots=args.slots)
    fifo = serve.run_open_loop(srv, fifo_reqs, policy="fifo")
    srv.close()
    log(f"bench served: batched, FIFO admission {fifo}")
    plain = serve.run_plain(plain_reqs)
    log(f"bench served: plain {plain}")
    mismatched = sum(int(a.best_len != b.best_len or not np.array_equal(a.best_tour, b.best_tour))
                     for a, b in zip(reqs, plain_reqs))
    mismatched += sum(int(a.best_len != b.best_len or not np.array_equal(a.best_tour, b.best_tour))
                      for a, b in zip(fifo_reqs, plain_reqs))
    rec = {
        "metric": "served solves/s and p99 latency (50 AS iterations per request)",
        "value": round(batched["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 0,
        "ms_per_step": round(batched["makespan_s"] * 1e3 / len(reqs), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(reqs)} requests, Poisson arrivals at 200/s, n log-uniform "
                               "in [100, 3000], m = n, uniform or 20-cluster layout (50/50), "
                               "alpha 1, beta 2, rho 0.5, 50 iterations each, per-request seed",
                   "requests": len(reqs), "rate_per_s": 200.0, "slots": args.slots,
                   "pool_bytes": pool},
        "latency_p50_s": round(batched["latency_p50_s"], 4),
        "latency_p99_s": round(batched["latency_p99_s"], 4),
        "admission": "size-aware: requests waiting under 10 s offered smallest solve first, "
                     "older ones first in arrival order",
        "batched": batched,
        "batched_fifo_admission": fifo,
        "plain_one_request_at_a_time": plain,
        "results_differing_from_plain": mismatched,
        "footprint_bytes_total": int(sum(footprint)),
        "footprint_formula_12n2_2mn_total": int(sum(formula)),
        "offered_load_note": "offered load exceeds device capacity; latency grows with trace length",
        "roofline": job_roofline(float(sum(construct_bytes(r.n, r.m) * r.iters for r in reqs)),
                                 batched["makespan_s"], len(reqs)),
    }
    return rec


ISOLATED_ANTS = 256  # one wavefront per compute unit, one per SIMD


def latency_floor(torch, aco, d, n: int, m_iso: int, con_ms: float) -> dict:
    """The construction step's latency with nothing to overlap it: the same
    instance with m_iso ants (at most one wavefront per compute unit), mean
    of 5 constructions after 2 iterations.  frac = that per-step time over
    the workload's own, i.e. how close the workload comes to the chain of
    dependent operations one step is."""
    col = aco.Colony(d, m_iso, ALPHA, BETA, RHO, seed=1)
    stream = torch.cuda.current_stream()
    for it in range(2):
        col.construct(it)
        col.update("gather")
    e0, e1 = _events(torch)
    torch.cuda.synchronize()
    e0.record(stream)
    for it in range(2, 7):
        col.construct(it)
    e1.record(stream)
    torch.cuda.synchronize()
    col.close()
    iso_ns = e0.elapsed_time(e1) / 5 * 1e6 / (n - 1)
    act_ns = con_ms * 1e6 / (n - 1)
    return {"ns_per_step_isolated": round(iso_ns, 1), "ants_isolated": m_iso,
            "ns_per_step": round(act_ns, 1), "frac": round(iso_ns / act_ns, 4),
            "note": (f"one construction step is a chain of dependent operations (row load, "
                     f"block sums, scans, pick); with {m_iso} ants no two wavefronts share a "
                     f"SIMD, so their per-step time is the chain's own latency, the bound "
                     f"of this latency-bound size; frac = that over this workload's "
                     f"per-step time")}


def run_single(args, torch, aco, name: str, steps: int, warmup: int, main: bool) -> dict:
    """One resident instance of WORKLOADS[name]: `warmup` untimed iterations,
    then `steps` timed iterations (construction, then the update of
    args.update), HIP events around every construction and update on the
    launch stream; then the other update variant on the same state.  The
    construction roofline is taken against the streaming read ceiling
    measured at the choice matrix's own footprint."""
    wl = WORKLOADS[name]
    n, m = wl["n"], wl["m"]
    _, d = tsp_inputs.instance(n, wl["layout"], side=wl["side"], seed=wl["seed"])
    col = aco.Colony(d, m, ALPHA, BETA, RHO, seed=1, atomic=True)
    stream = torch.cuda.current_stream()
    log(f"bench: {name} n={n} m={m} {col.describe()}")

    it = 0
    for _ in range(warmup):
        col.construct(it)
        launched(torch)
        col.update(args.update)
        launched(torch)
        it += 1
    torch.cuda.synchronize()

    K = steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        ev[3 * s].record(stream)
        col.construct(it)
        launched(torch)
        ev[3 * s + 1].record(stream)
        col.update(args.update)
        launched(torch)
        ev[3 * s + 2].record(stream)
        it += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_con = np.array([ev[3 * s].elapsed_time(ev[3 * s + 1]) for s in range(K)])
    t_upd = np.array([ev[3 * s + 1].elapsed_time(ev[3 * s + 2]) for s in range(K)])
    log(f"bench: {name}: timed {K} steps in {wall:.3f} s")
    tours, _ = col.tours()
    tile = int(col.describe().split("cities_per_lane=")[1].split()[0])

    # the other update variants, timed after the timed region on the same state
    t_other = {}
    for kind in ("gather", "atomic", "atomic_direct"):
        if kind == args.update:
            continue
        t_other[kind] = []
        for _ in range(max(3, min(K, 10))):
            col.construct(it)
            launched(torch)
            e0, e1 = _events(torch)
            e0.record(stream)
            col.update(kind)
            launched(torch)
            e1.record(stream)
            torch.cuda.synchronize()
            t_other[kind].append(e0.elapsed_time(e1))
            it += 1
    t_upd_v = {args.update: float(t_upd.mean())}
    t_upd_v.update({k: float(np.mean(v)) for k, v in t_other.items()})
    best_tour, best_len = col.best()
    col.close()

    ld = (n + 63) // 64 * 64
    ant_steps = m * (n - 1)
    ms_step = wall * 1e3 / K
    con_ms = float(t_con.mean())
    alg = construct_bytes(n, m)
    achieved = alg / (con_ms * 1e-3) / 1e9
    passes = (n + 64 * tile - 1) // (64 * tile)
    req = requested_bytes(tours, n, skip=passes >= 3)
    foot = n * ld * 4
    ceil = stream_read_ceiling(torch, aco, foot)
    rows_ceil = random_rows_ceiling(torch, aco, n, m)
    peak = max(ceil["GBps"], rows_ceil["GBps"])
    roofline = {"bound": "mall" if foot > (4 << 20) else "l2", "achieved": round(achieved, 1),
                "peak": peak, "unit": "GB/s", "frac": round(achieved / peak, 4),
                "traffic": None, "kernel": f"k_construct<{tile},{passes}>",
                "algorithmic_bytes_per_launch": alg,
                "peak_note": (f"measured at the choice matrix's {foot / 1e6:.1f} MB footprint, "
                              f"the better of two reads of it: a streaming read, every XCD "
                              f"walking all of it, best of {len(PROBE_SHAPES)} load shapes "
                              f"(aco_probe_read_shape: {ceil['GBps']} GB/s with "
                              f"{ceil['loads_in_flight']} loads in flight"
                              f"{', nontemporal' if ceil['nontemporal'] else ''}, "
                              f"{ceil['reps']} passes, {ceil['ms']} ms), and random whole rows "
                              f"with 1, 2, 4 and 8 times the kernel's {m} wavefronts and one or "
                              f"two rows in flight each (aco_probe_rows_shape: "
                              f"{rows_ceil['GBps']} GB/s with wavefronts x rows in flight = "
                              f"{rows_ceil['shape']}), where each XCD's L2 keeps a share of the "
                              f"rows as it does for the kernel"),
                "peak_stream_GBps": ceil["GBps"],
                "peak_by_shape_GBps": ceil["by_shape_GBps"],
                "peak_random_rows_GBps": rows_ceil["GBps"],
                "peak_random_rows_by_shape_GBps": rows_ceil["by_shape_GBps"],
                "hbm_peak": HBM_PEAK_GBPS, "frac_of_hbm_peak": round(achieved / HBM_PEAK_GBPS, 4),
                "requested_bytes_per_launch": req,
                "requested_GBps": round(req / (con_ms * 1e-3) / 1e9, 1),
                "frac_requested": round(req / (con_ms * 1e-3) / 1e9 / peak, 4)}
    if passes >= 3:
        roofline["frac_note"] = (
            f"achieved counts the whole {n}-city row per ant-step (4n bytes), but the kernel "
            f"does not load a 16-byte group of cities once all four are visited, so it requests "
            f"only {req / alg:.3f} of those bytes: frac can reach 1 while the bytes it moves "
            f"(frac_requested, and the counter bytes past L2 in frac_traffic_of_stream) stay "
            f"below the measured ceiling")
    if main:
        traffic, traffic_note = traffic_from_profile()
        roofline["traffic"] = traffic
        roofline["traffic_note"] = traffic_note
        if traffic:
            # the bytes that crossed from the Infinity Cache / HBM side, against
            # the sweep, which the L2 does not filter either
            tr = traffic / (con_ms * 1e-3) / 1e9
            roofline["traffic_GBps"] = round(tr, 1)
            roofline["frac_traffic_of_stream"] = round(tr / ceil["GBps"], 4)

    upd = {}
    for kind, ms in t_upd_v.items():
        b = UPDATE_BYTES[kind](n, m)
        upd[kind] = {"ms": round(ms, 4), "algorithmic_bytes": b,
                     "GBps": round(b / (ms * 1e-3) / 1e9, 1)}
    rec = {
        "metric": METRIC,
        "value": round(ant_steps / (ms_step * 1e-3), 1),
        "unit": "ant-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"Ant System, n={n} cities {wl['layout']} in "
                               f"[0,{wl['side']}]^2 (instance seed {wl['seed']}), m={m} ants, "
                               f"alpha={ALPHA}, beta={BETA}, rho={RHO}, Philox seed 1, "
                               f"{args.update} update; one step = one iteration",
                   "n": n, "m": m, "layout": wl["layout"], "update": args.update},
        "construct_ms": round(con_ms, 4),
        "construct_ant_steps_per_s": round(ant_steps / (con_ms * 1e-3), 1),
        "update": upd,
        "best_len_after_run": int(best_len),
        "roofline": roofline,
    }
    if roofline["bound"] == "l2" and m > ISOLATED_ANTS and not args.no_latency_floor:
        # latency-bound sizes (the matrix within one XCD's L2): the step chain's
        # own latency, measured with few enough ants that no two share a SIMD
        rec["latency_floor"] = latency_floor(torch, aco, d, n, ISOLATED_ANTS, con_ms)
    if main:
        # each update kernel against a copy of its own footprint (one launch)
        for kind in upd:
            b = upd[kind]["algorithmic_bytes"]
            cc = copy_ceiling(torch, aco, b)
            upd[kind]["roofline"] = {
                "bound": "mall" if b < (256 << 20) else "hbm", "achieved": upd[kind]["GBps"],
                "peak": cc["GBps"], "unit": "GB/s",
                "frac": round(upd[kind]["GBps"] / cc["GBps"], 4),
                "peak_note": (f"measured: one aco_probe_copy launch over {b / 1e6:.1f} MB (half "
                              f"read, half written), mean of 20 launches, "
                              f"{cc['ms_per_launch']} ms each"),
                "hbm_peak": HBM_PEAK_GBPS,
                "frac_of_hbm_peak": round(upd[kind]["GBps"] / HBM_PEAK_GBPS, 4)}
    return rec, d


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["batch256", "served", "all"],
                    default="all",
                    help="all (default): the n = 2400 line with every other workload as a "
                         "sub-record; otherwise that workload alone")
    ap.add_argument("--requests", type=int, default=100, help="served workload: trace length")
    ap.add_argument("--slots", type=int, default=32, help="served workload: server slots")
    ap.add_argument("--update", choices=["gather", "atomic", "atomic_direct"], default="gather")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="host time budget of the oracle sample (0 skips it)")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the HBM and 160 MB streaming probes and the random-row probes")
    ap.add_argument("--sync-launches", action="store_true",
                    help="synchronise with the host after every launch (for profiled runs; "
                         "ms_per_step then includes the round trips)")
    ap.add_argument("--no-product", action="store_true",
                    help="skip the product-and-argmax construction block")
    ap.add_argument("--no-latency-floor", action="store_true",
                    help="skip the isolated-chain timing of the L2-resident workloads (for "
                         "profiled runs, whose per-kernel statistics would otherwise mix in "
                         "its smaller launches)")
    ap.add_argument("--nn", type=int, default=30,
                    help="also time candidate-list construction with lists of this length "
                         "(0 skips it)")
    args = ap.parse_args()

    global SYNC_LAUNCHES
    SYNC_LAUNCHES = args.sync_launches
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1 "
                                   "(the design notes describe how the path would shard)"}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    from paper_1101_2678_amd import aco

    if args.workload == "batch256":
        print(json.dumps(bench_batch(args, torch, aco)), flush=True)
        return
    if args.workload == "served":
        print(json.dumps(bench_served(args, torch, aco)), flush=True)
        return
    if args.workload not in ("all", "n2400"):
        rec, _ = run_single(args, torch, aco, args.workload, args.steps, args.warmup, main=False)
        print(json.dumps(rec), flush=True)
        return

    rec, d = run_single(args, torch, aco, "n2400", args.steps, args.warmup, main=True)
    n, m = rec["config"]["n"], rec["config"]["m"]
    # a plain copy of known size: profiled runs calibrate FETCH_SIZE and
    # WRITE_SIZE on it
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    aco.probe_copy(dst, src)
    torch.cuda.synchronize()
    rec["copy_calibration_bytes"] = src.numel() * 4
    del src, dst
    if not args.no_probe:
        log("bench: HBM and 160 MB streaming probes, random-row probes")
        rec["probe"] = {
            "stream_read_4GiB": stream_read_ceiling(torch, aco, 4 << 30),
            "stream_read_160MB": stream_read_ceiling(torch, aco, 160 << 20),
            "random_rows_same_footprint_GBps": random_rows_rate(torch, aco, n, m, n),
            "random_rows_160MB_GBps": random_rows_rate(torch, aco, n, m,
                                                       (160 << 20) // (4 * ((n + 63) // 64 * 64))),
            "hbm_peak_GBps": HBM_PEAK_GBPS,
        }
    if not args.no_product:
        log("bench: product-and-argmax construction")
        rec["product"] = bench_product(torch, aco, d, m, args.steps, args.warmup, args.update,
                                       min(3.0, args.cpu_seconds))
    if args.nn > 0:
        log(f"bench: candidate-list construction, nn={args.nn}")
        rec["nn_list"] = bench_nn(torch, aco, d, m, args.nn, args.steps, args.warmup,
                                  args.update, min(3.0, args.cpu_seconds))
    if args.workload == "all":
        configs = rec["configs"] = run_configs(args, torch, aco)
        srv = configs["served"]
        rec["served_solves_per_s"] = srv["value"]
        rec["served_latency_p50_s"] = srv["latency_p50_s"]
        rec["served_latency_p99_s"] = srv["latency_p99_s"]
        rec["served_plain_solves_per_s"] = round(
            srv["plain_one_request_at_a_time"]["solves_per_s"], 3)
        rec["served_plain_latency_p99_s"] = round(
            srv["plain_one_request_at_a_time"]["latency_p99_s"], 4)
        rec["batch256_solves_per_s"] = configs["batch256"]["value"]
        rec["batch256_one_per_launch_solves_per_s"] = (
            configs["batch256"]["one_instance_per_launch"]["solves_per_s"])
    if args.cpu_seconds > 0:
        log(f"bench: timing the oracle (up to ~{args.cpu_seconds:.0f} s of host work)")
        rec["cpu_baseline"] = cpu_baseline(d, m, args.cpu_seconds)
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)


def run_configs(args, torch, aco) -> dict:
    """Every workload other than n = 2400, as sub-records of the main line."""
    configs = {}
    for name in ("n100", "n1000u", "n1000c"):
        configs[name], _ = run_single(args, torch, aco, name, args.steps, args.warmup,
                                      main=False)
    log("bench: batch256")
    configs["batch256"] = bench_batch(args, torch, aco)
    log("bench: served")
    configs["served"] = bench_served(args, torch, aco)
    return configs


if __name__ == "__main__":
    main()
