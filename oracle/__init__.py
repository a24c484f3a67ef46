"""Serial CPU oracle for the Ant System on the symmetric TSP (arXiv:1101.2678).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never takes an input that the HIP library
produced.

The arithmetic lives in ``aco_oracle.c`` (plain serial C); this module only
marshals numpy arrays through ctypes and strings the per-iteration calls
together in the order of Section II: construct all tours, keep the
best-so-far, then update the pheromone (evaporate, deposit, refresh choice).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "aco_oracle.c")]
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (no FP contraction, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", *CFLAGS, "-o", tmp, *SOURCES, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None

_u16p = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(LIB_PATH)
        c = ctypes
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_draw.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32, c.c_uint32]
        L.oracle_draw.restype = c.c_uint32
        L.oracle_uniform.argtypes = [c.c_uint32]
        L.oracle_uniform.restype = c.c_float
        L.oracle_start_city.argtypes = [c.c_uint32, c.c_int32]
        L.oracle_start_city.restype = c.c_int32
        L.oracle_heur.argtypes = [c.c_int32, c.c_int32]
        L.oracle_heur.restype = c.c_float
        L.oracle_choice.argtypes = [c.c_int32, _f32p, _i32p, c.c_int32, c.c_int32, _f32p]
        L.oracle_choice.restype = None
        L.oracle_nn_tour_length.argtypes = [c.c_int32, _i32p]
        L.oracle_nn_tour_length.restype = c.c_int64
        L.oracle_init.argtypes = [c.c_int32, c.c_int32, _i32p, c.c_int32, c.c_int32,
                                  _f32p, _f32p, c.POINTER(c.c_float)]
        L.oracle_init.restype = None
        L.oracle_s64.argtypes = [_f32p, _f32p]
        L.oracle_s64.restype = None
        L.oracle_r64_select.argtypes = [c.c_int32, _f32p, _u8p, c.c_float]
        L.oracle_r64_select.restype = c.c_int32
        L.oracle_r64_select_batch.argtypes = [c.c_int32, c.c_int32, _f32p, _u8p, _f32p, _i32p]
        L.oracle_r64_select_batch.restype = None
        L.oracle_construct_ant.argtypes = [c.c_int32, _f32p, _i32p, c.c_uint64, c.c_uint32,
                                           c.c_uint32, _u16p]
        L.oracle_construct_ant.restype = c.c_int64
        L.oracle_nn_lists.argtypes = [c.c_int32, _i32p, c.c_int32, _u16p]
        L.oracle_nn_lists.restype = None
        L.oracle_construct_ant_nn.argtypes = [c.c_int32, _f32p, _i32p, _u16p, c.c_int32,
                                              c.c_uint64, c.c_uint32, c.c_uint32, _u16p]
        L.oracle_construct_ant_nn.restype = c.c_int64
        L.oracle_product_uniform.argtypes = [c.c_uint64, c.c_uint32, c.c_uint32, c.c_uint32,
                                             c.c_int32]
        L.oracle_product_uniform.restype = c.c_float
        L.oracle_product_select.argtypes = [c.c_int32, _f32p, _u8p, _f32p]
        L.oracle_product_select.restype = c.c_int32
        L.oracle_product_select_batch.argtypes = [c.c_int32, c.c_int32, _f32p, _u8p, _f32p,
                                                  _i32p]
        L.oracle_product_select_batch.restype = None
        L.oracle_construct_ant_product.argtypes = [c.c_int32, _f32p, _i32p, c.c_uint64,
                                                   c.c_uint32, c.c_uint32, _u16p]
        L.oracle_construct_ant_product.restype = c.c_int64
        L.oracle_construct.argtypes = [c.c_int32, c.c_int32, _f32p, _i32p, c.c_uint64,
                                       c.c_uint32, _u16p, _i64p]
        L.oracle_construct.restype = None
        L.oracle_deposit_amount.argtypes = [c.c_int64]
        L.oracle_deposit_amount.restype = c.c_float
        L.oracle_deposit.argtypes = [c.c_int32, c.c_int32, _u16p, _i64p, _f64p]
        L.oracle_deposit.restype = c.c_int32
        L.oracle_update.argtypes = [c.c_int32, c.c_int32, c.c_float, _u16p, _i64p, _i32p,
                                    c.c_int32, c.c_int32, _f32p, _f32p]
        L.oracle_update.restype = c.c_int32
        L.oracle_best_of.argtypes = [c.c_int32, _i64p, c.POINTER(c.c_int64)]
        L.oracle_best_of.restype = c.c_int32
        _lib = L
    return _lib


# ---------------------------------------------------------------- thin wrappers
def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def draw(seed: int, it: int, ant: int, step: int) -> int:
    return int(lib().oracle_draw(seed, it, ant, step))


def uniform(x0: int) -> float:
    return float(lib().oracle_uniform(x0))


def start_city(x0: int, n: int) -> int:
    return int(lib().oracle_start_city(x0, n))


def heur(d: int, beta: int) -> np.float32:
    return np.float32(lib().oracle_heur(int(d), int(beta)))


def choice(tau: np.ndarray, dist: np.ndarray, alpha: int, beta: int) -> np.ndarray:
    n = dist.shape[0]
    out = np.empty((n, n), np.float32)
    lib().oracle_choice(n, np.ascontiguousarray(tau, np.float32),
                        np.ascontiguousarray(dist, np.int32), alpha, beta, out)
    return out


def nn_tour_length(dist: np.ndarray) -> int:
    return int(lib().oracle_nn_tour_length(dist.shape[0], np.ascontiguousarray(dist, np.int32)))


def s64(x) -> np.ndarray:
    out = np.empty(64, np.float32)
    lib().oracle_s64(np.ascontiguousarray(x, np.float32), out)
    return out


def r64_select(row, feasible, u: float) -> int:
    row = np.ascontiguousarray(row, np.float32)
    feas = np.ascontiguousarray(feasible, np.uint8)
    return int(lib().oracle_r64_select(row.shape[0], row, feas, np.float32(u)))


def r64_select_batch(rows, feasible, u) -> np.ndarray:
    rows = np.ascontiguousarray(rows, np.float32)
    count, n = rows.shape
    out = np.empty(count, np.int32)
    lib().oracle_r64_select_batch(n, count, rows, np.ascontiguousarray(feasible, np.uint8),
                                  np.ascontiguousarray(u, np.float32), out)
    return out


def construct_ant(choice_m: np.ndarray, dist: np.ndarray, seed: int, it: int, ant: int):
    n = dist.shape[0]
    tour = np.empty(n + 1, np.uint16)
    length = lib().oracle_construct_ant(n, np.ascontiguousarray(choice_m, np.float32),
                                        np.ascontiguousarray(dist, np.int32), seed, it, ant,
                                        tour)
    return tour, int(length)


def product_uniform(seed: int, it: int, ant: int, step: int, j: int) -> float:
    return float(lib().oracle_product_uniform(seed, it, ant, step, j))


def product_select(row, feasible, r) -> int:
    row = np.ascontiguousarray(row, np.float32)
    return int(lib().oracle_product_select(row.shape[0], row,
                                           np.ascontiguousarray(feasible, np.uint8),
                                           np.ascontiguousarray(r, np.float32)))


def product_select_batch(rows, feasible, r) -> np.ndarray:
    rows = np.ascontiguousarray(rows, np.float32)
    count, n = rows.shape
    out = np.empty(count, np.int32)
    lib().oracle_product_select_batch(count, n, rows, np.ascontiguousarray(feasible, np.uint8),
                                      np.ascontiguousarray(r, np.float32), out)
    return out


def construct_ant_product(choice_m, dist, seed: int, it: int, ant: int):
    n = dist.shape[0]
    tour = np.empty(n + 1, np.uint16)
    length = lib().oracle_construct_ant_product(n, np.ascontiguousarray(choice_m, np.float32),
                                                np.ascontiguousarray(dist, np.int32), seed, it,
                                                ant, tour)
    return tour, int(length)


def construct_product(choice_m, dist, m: int, seed: int, it: int, threads: int = 1):
    """All m product-rule tours of iteration ``it`` (each ant one serial call)."""
    n = dist.shape[0]
    tours = np.empty((m, n + 1), np.uint16)
    lens = np.empty(m, np.int64)

    def one(k):
        t, ln = construct_ant_product(choice_m, dist, seed, it, k)
        tours[k] = t
        lens[k] = ln

    if threads <= 1:
        for k in range(m):
            one(k)
    else:
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, range(m)))
    return tours, lens


def nn_lists(dist: np.ndarray, nn: int) -> np.ndarray:
    n = dist.shape[0]
    out = np.empty((n, nn), np.uint16)
    lib().oracle_nn_lists(n, np.ascontiguousarray(dist, np.int32), nn, out)
    return out


def construct_ant_nn(choice_m, dist, nnl, seed: int, it: int, ant: int):
    n = dist.shape[0]
    nnl = np.ascontiguousarray(nnl, np.uint16)
    tour = np.empty(n + 1, np.uint16)
    length = lib().oracle_construct_ant_nn(n, np.ascontiguousarray(choice_m, np.float32),
                                           np.ascontiguousarray(dist, np.int32), nnl,
                                           nnl.shape[1], seed, it, ant, tour)
    return tour, int(length)


def construct_nn(choice_m, dist, nnl, m: int, seed: int, it: int, threads: int = 1):
    """All m nn-list tours of iteration ``it`` (each ant one serial call)."""
    n = dist.shape[0]
    tours = np.empty((m, n + 1), np.uint16)
    lens = np.empty(m, np.int64)

    def one(k):
        t, ln = construct_ant_nn(choice_m, dist, nnl, seed, it, k)
        tours[k] = t
        lens[k] = ln

    if threads <= 1:
        for k in range(m):
            one(k)
    else:
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, range(m)))
    return tours, lens


def construct(choice_m: np.ndarray, dist: np.ndarray, m: int, seed: int, it: int,
              threads: int = 1):
    """All m tours of iteration ``it``.  With threads > 1 the ants are split
    over Python threads (ctypes releases the GIL); every ant is still the
    same serial call, so the result does not depend on ``threads``."""
    n = dist.shape[0]
    tours = np.empty((m, n + 1), np.uint16)
    lens = np.empty(m, np.int64)
    choice_c = np.ascontiguousarray(choice_m, np.float32)
    dist_c = np.ascontiguousarray(dist, np.int32)
    if threads <= 1:
        lib().oracle_construct(n, m, choice_c, dist_c, seed, it, tours, lens)
        return tours, lens
    from concurrent.futures import ThreadPoolExecutor

    def one(k):
        row = np.empty(n + 1, np.uint16)
        ln = lib().oracle_construct_ant(n, choice_c, dist_c, seed, it, k, row)
        tours[k] = row
        lens[k] = ln

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, range(m)))
    return tours, lens


def deposit_amount(length: int) -> np.float32:
    return np.float32(lib().oracle_deposit_amount(int(length)))


def deposit(tours: np.ndarray, lens: np.ndarray, n: int):
    m = tours.shape[0]
    D = np.empty((n, n), np.float64)
    st = lib().oracle_deposit(n, m, np.ascontiguousarray(tours, np.uint16),
                              np.ascontiguousarray(lens, np.int64), D)
    return D, int(st)


def update(tau: np.ndarray, tours: np.ndarray, lens: np.ndarray, dist: np.ndarray,
           rho: float, alpha: int, beta: int):
    """Returns (tau', choice').  Raises if the exactness condition fails."""
    n = dist.shape[0]
    m = tours.shape[0]
    tau2 = np.array(tau, np.float32, copy=True, order="C")
    ch = np.empty((n, n), np.float32)
    st = lib().oracle_update(n, m, np.float32(rho), np.ascontiguousarray(tours, np.uint16),
                             np.ascontiguousarray(lens, np.int64),
                             np.ascontiguousarray(dist, np.int32), alpha, beta, tau2, ch)
    if st != 0:
        raise RuntimeError(f"oracle_update status {st}")
    return tau2, ch


@dataclass
class OracleState:
    """The AS state after some iterations: tau, choice and the best tour."""
    n: int
    m: int
    alpha: int
    beta: int
    rho: float
    seed: int
    tau: np.ndarray
    choice: np.ndarray
    tau0: float
    it: int = 0
    best_len: int = 2**62
    best_tour: np.ndarray | None = None
    history: list = field(default_factory=list)


def init(dist: np.ndarray, m: int, alpha: int, beta: int, rho: float, seed: int) -> OracleState:
    n = dist.shape[0]
    tau = np.empty((n, n), np.float32)
    ch = np.empty((n, n), np.float32)
    t0 = ctypes.c_float()
    lib().oracle_init(n, m, np.ascontiguousarray(dist, np.int32), alpha, beta, tau, ch,
                      ctypes.byref(t0))
    return OracleState(n, m, alpha, beta, rho, seed, tau, ch, float(t0.value))


def iterate(st: OracleState, dist: np.ndarray, threads: int = 1, keep: bool = False,
            nnl: np.ndarray | None = None, rule: str = "r64"):
    """One AS iteration: construct (Section II; over the candidate lists
    ``nnl`` if given; rule "product": the product-and-argmax selection of
    Section III-A), best-so-far, update (Eqs. 2-4)."""
    if nnl is not None:
        tours, lens = construct_nn(st.choice, dist, nnl, st.m, st.seed, st.it, threads)
    elif rule == "product":
        tours, lens = construct_product(st.choice, dist, st.m, st.seed, st.it, threads)
    else:
        tours, lens = construct(st.choice, dist, st.m, st.seed, st.it, threads)
    best = ctypes.c_int64(st.best_len)
    who = lib().oracle_best_of(st.m, lens, ctypes.byref(best))
    if who >= 0:
        st.best_len = int(best.value)
        st.best_tour = tours[who].copy()
    tau_before = st.tau.copy() if keep else None
    st.tau, st.choice = update(st.tau, tours, lens, dist, st.rho, st.alpha, st.beta)
    if keep:
        st.history.append(dict(it=st.it, tours=tours, lens=lens, tau_before=tau_before,
                               tau_after=st.tau.copy()))
    st.it += 1
    return tours, lens


def solve(dist: np.ndarray, m: int, alpha: int, beta: int, rho: float, seed: int,
          iters: int, threads: int = 1, keep: bool = False, nn: int | None = None,
          rule: str = "r64") -> OracleState:
    """``iters`` iterations from the initial state; nn: candidate-list
    construction with lists of that length; rule: "r64" or "product"."""
    st = init(dist, m, alpha, beta, rho, seed)
    nnl = None if nn is None else nn_lists(dist, nn)
    for _ in range(iters):
        iterate(st, dist, threads, keep, nnl, rule)
    return st
