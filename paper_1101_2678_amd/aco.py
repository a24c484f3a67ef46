"""ctypes binding of libaco (include/aco.h).

Argument marshalling only: every step of the Ant System runs in the HIP
kernels of libaco.so.  torch provides the device workspace and the stream.
If libaco.so is missing, importing this module raises; nothing falls back to
a CPU path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libaco.so")

ACO_OK, ACO_ERR_INVALID, ACO_ERR_NOMEM, ACO_ERR_DEVICE, ACO_ERR_STATE = range(5)
GATHER, ATOMIC, ATOMIC_DIRECT = 0, 1, 2
_KIND = {"gather": GATHER, "atomic": ATOMIC, "atomic_direct": ATOMIC_DIRECT, GATHER: GATHER,
         ATOMIC: ATOMIC, ATOMIC_DIRECT: ATOMIC_DIRECT}


class AcoError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class BatchConfig(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_int32), ("tile4_max_n", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("alpha", ctypes.c_int32),
                ("beta", ctypes.c_int32), ("rho", ctypes.c_float), ("seed", ctypes.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1101_2678_amd._build` "
            "(or __graft_entry__.build()); there is no CPU fallback")
    # libaco.so needs the HIP runtime torch ships.  Loaded before torch, the
    # dynamic linker would take the system's copy instead (torch's directory
    # has it under another file name), and torch would then load its own: two
    # runtimes in one process, the library's seeing no device.  With torch
    # loaded first, the library binds to torch's runtime.
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp, sz, i32, u32, i64 = c.c_void_p, c.c_size_t, c.c_int32, c.c_uint32, c.c_int64
    sigs = {
        "aco_workspace_bytes": (sz, [c.POINTER(Params), i32]),
        "aco_init": (i32, [c.POINTER(vp), c.POINTER(Params), vp, vp, sz, vp]),
        "aco_construct": (i32, [vp, u32]),
        "aco_update": (i32, [vp, i32]),
        "aco_update_atomic_noalloc": (i32, [vp]),
        "aco_solve": (i32, [vp, u32, i32, vp, vp]),
        "aco_read_tours": (i32, [vp, vp, vp]),
        "aco_construct_product": (i32, [vp, u32]),
        "aco_solve_product": (i32, [vp, u32, i32, vp, vp]),
        "aco_test_product_select": (i32, [i32, i32, vp, vp, vp, vp, vp]),
        "aco_nn_workspace_bytes": (sz, [i32, i32]),
        "aco_nn_attach": (i32, [vp, i32, vp, sz]),
        "aco_construct_nn": (i32, [vp, u32]),
        "aco_solve_nn": (i32, [vp, u32, i32, vp, vp]),
        "aco_read_nn_lists": (i32, [vp, vp]),
        "aco_read_tau": (i32, [vp, vp]),
        "aco_read_choice": (i32, [vp, vp]),
        "aco_read_best": (i32, [vp, vp, vp]),
        "aco_restore": (i32, [vp, vp, u32, i64, vp]),
        "aco_get_iter": (i32, [vp, c.POINTER(u32)]),
        "aco_sync": (i32, [vp]),
        "aco_destroy": (None, [vp]),
        "aco_status_str": (c.c_char_p, [i32]),
        "aco_last_error": (c.c_char_p, []),
        "aco_describe": (i32, [vp, c.c_char_p, sz]),
        "aco_test_select": (i32, [i32, i32, i32, vp, vp, vp, vp, vp]),
        "aco_test_select_shape": (i32, [i32, i32, i32, i32, vp, vp, vp, vp, vp]),
        "aco_set_tile": (i32, [i32, i32, i32]),
        "aco_set_shape": (i32, [i32, i32, i32, i32]),
        "aco_get_tile": (i32, [i32]),
        "aco_get_waves": (i32, [i32]),
        "aco_reset_tiles": (None, []),
        "aco_autotune": (i32, [vp, sz, vp, i32, i32, vp, vp, vp, vp]),
        "aco_batch_workspace_bytes": (sz, [i32, vp]),
        "aco_batch_init": (i32, [c.POINTER(vp), i32, vp, vp, vp, sz, vp]),
        "aco_batch_run": (i32, [vp, u32, i32]),
        "aco_batch_read_best": (i32, [vp, i32, vp, vp]),
        "aco_batch_read_tours": (i32, [vp, i32, vp, vp]),
        "aco_batch_read_tau": (i32, [vp, i32, vp]),
        "aco_batch_get_iter": (i32, [vp, i32, c.POINTER(u32)]),
        "aco_batch_sync": (i32, [vp]),
        "aco_batch_set_config": (i32, [vp, c.POINTER(BatchConfig)]),
        "aco_batch_get_config": (i32, [vp, c.POINTER(BatchConfig)]),
        "aco_batch_autotune": (i32, [vp, vp, i32, u32, c.POINTER(i32), vp]),
        "aco_batch_destroy": (None, [vp]),
        "aco_server_table_bytes": (sz, [i32, i32, i32, i32]),
        "aco_server_create": (i32, [c.POINTER(vp), vp, sz, i32, i32, i32, i32, vp]),
        "aco_server_submit": (i32, [vp, c.POINTER(Params), vp, u32, i64, c.POINTER(i32)]),
        "aco_server_step": (i32, [vp, c.POINTER(i32)]),
        "aco_server_collect": (i32, [vp, vp, vp, i32, c.POINTER(i32)]),
        "aco_server_result": (i32, [vp, i32, vp, vp]),
        "aco_server_read_tau": (i32, [vp, i32, vp]),
        "aco_server_release": (i32, [vp, i32]),
        "aco_server_stats": (i32, [vp, c.POINTER(i32), c.POINTER(i32), c.POINTER(i32),
                                   c.POINTER(sz), c.POINTER(sz), c.POINTER(c.c_uint64)]),
        "aco_server_destroy": (None, [vp]),
        "aco_probe_copy": (i32, [vp, vp, sz, vp]),
        "aco_probe_read": (i32, [vp, sz, i32, vp, vp]),
        "aco_probe_read_shape": (i32, [vp, sz, i32, i32, i32, vp, vp]),
        "aco_probe_rows": (i32, [vp, i32, i32, i32, i32, i32, vp, vp]),
        "aco_probe_rows_shape": (i32, [vp, i32, i32, i32, i32, i32, i32, vp, vp]),
        "aco_probe_philox": (i32, [i32, i32, u32, vp, vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def _check(status: int, where: str):
    if status != ACO_OK:
        detail = (lib.aco_last_error() or b"").decode() or lib.aco_status_str(status).decode()
        raise AcoError(status, where, detail)


def _stream_handle(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def workspace_bytes(n: int, m: int, alpha: int = 1, beta: int = 2, rho: float = 0.5,
                    seed: int = 1, atomic: bool = True) -> int:
    p = Params(n, m, alpha, beta, rho, seed)
    return int(lib.aco_workspace_bytes(ctypes.byref(p), 1 if atomic else 0))


def as_dist(dist) -> np.ndarray:
    """The distance matrix as the library takes it: square, C-contiguous
    int32.  Integer input outside the int32 range and non-integer input are
    refused rather than cast, so that no distance changes on the way in (the
    library checks symmetry, the diagonal and the range itself)."""
    a = np.asarray(dist)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("dist must be a square matrix")
    if not np.issubdtype(a.dtype, np.integer):
        raise TypeError(f"dist must hold integers (nint distances), not {a.dtype}")
    if a.size and (int(a.min()) < np.iinfo(np.int32).min or int(a.max()) > np.iinfo(np.int32).max):
        raise ValueError("dist values must fit int32")
    return np.ascontiguousarray(a, dtype=np.int32)


class Colony:
    """One Ant System instance resident on a GPU.

    dist: (n, n) int32 symmetric distance matrix (host numpy array).
    The device workspace is a torch uint8 tensor; all kernels run on `stream`
    (default: torch's current stream on `device`).
    """

    def __init__(self, dist, m: int, alpha: int = 1, beta: int = 2, rho: float = 0.5,
                 seed: int = 1, atomic: bool = True, device="cuda", stream=None):
        import torch

        d = as_dist(dist)
        self.n, self.m = int(d.shape[0]), int(m)
        self.params = Params(self.n, self.m, alpha, beta, rho, seed)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.atomic = bool(atomic)
        nbytes = lib.aco_workspace_bytes(ctypes.byref(self.params), 1 if atomic else 0)
        if nbytes == 0:
            _check(ACO_ERR_INVALID, "aco_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        # the kernels use the workspace on self.stream: the caching allocator
        # must not reuse it before the work queued there has finished
        self.workspace.record_stream(self.stream)
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.aco_init(ctypes.byref(self._ctx), ctypes.byref(self.params),
                                d.ctypes.data_as(ctypes.c_void_p),
                                ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                _stream_handle(self.stream)), "aco_init")

    # ---- asynchronous steps
    def construct(self, it: int):
        _check(lib.aco_construct(self._ctx, it), "aco_construct")

    def attach_nn(self, nn: int = 30):
        """Builds candidate lists of length nn on the device (see
        aco_nn_attach); the tables live in a workspace of their own."""
        import torch

        nbytes = int(lib.aco_nn_workspace_bytes(self.n, nn))
        if nbytes == 0:
            _check(ACO_ERR_INVALID, "aco_nn_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ws.record_stream(self.stream)
        _check(lib.aco_nn_attach(self._ctx, nn, ctypes.c_void_p(ws.data_ptr()), nbytes),
               "aco_nn_attach")
        self.nn_workspace, self.nn = ws, int(nn)

    def construct_product(self, it: int):
        _check(lib.aco_construct_product(self._ctx, it), "aco_construct_product")

    def construct_nn(self, it: int):
        _check(lib.aco_construct_nn(self._ctx, it), "aco_construct_nn")

    def nn_lists(self):
        out = np.empty((self.n, self.nn), np.uint16)
        _check(lib.aco_read_nn_lists(self._ctx, out.ctypes.data_as(ctypes.c_void_p)),
               "aco_read_nn_lists")
        return out

    def update(self, kind="gather"):
        _check(lib.aco_update(self._ctx, _KIND[kind]), "aco_update")

    def update_atomic_noalloc(self):
        """The atomic update with the library's static deposit matrix
        (aco_update_atomic_noalloc: n <= 1024, no workspace part needed)."""
        _check(lib.aco_update_atomic_noalloc(self._ctx), "aco_update_atomic_noalloc")

    # ---- synchronous calls
    def solve(self, iters: int, kind="gather", rule: str = "r64"):
        """rule "r64": full-row construction; "nn": candidate lists (needs
        attach_nn); "product": the paper's product-and-argmax selection."""
        fn = {"r64": lib.aco_solve, "nn": lib.aco_solve_nn, "product": lib.aco_solve_product}[rule]
        tour = np.empty(self.n + 1, np.uint16)
        length = ctypes.c_int64()
        _check(fn(self._ctx, iters, _KIND[kind], tour.ctypes.data_as(ctypes.c_void_p),
                  ctypes.byref(length)), fn.__name__)
        return tour, int(length.value)

    def tours(self):
        t = np.empty((self.m, self.n + 1), np.uint16)
        ln = np.empty(self.m, np.int64)
        _check(lib.aco_read_tours(self._ctx, t.ctypes.data_as(ctypes.c_void_p),
                                  ln.ctypes.data_as(ctypes.c_void_p)), "aco_read_tours")
        return t, ln

    def tau(self):
        out = np.empty((self.n, self.n), np.float32)
        _check(lib.aco_read_tau(self._ctx, out.ctypes.data_as(ctypes.c_void_p)), "aco_read_tau")
        return out

    def choice(self):
        out = np.empty((self.n, self.n), np.float32)
        _check(lib.aco_read_choice(self._ctx, out.ctypes.data_as(ctypes.c_void_p)),
               "aco_read_choice")
        return out

    def best(self):
        tour = np.empty(self.n + 1, np.uint16)
        length = ctypes.c_int64()
        _check(lib.aco_read_best(self._ctx, tour.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(length)), "aco_read_best")
        return tour, int(length.value)

    def restore(self, tau, it: int, best_len: int = -1, best_tour=None):
        t = np.ascontiguousarray(tau, np.float32)
        bt = None if best_tour is None else np.ascontiguousarray(best_tour, np.uint16)
        _check(lib.aco_restore(self._ctx, t.ctypes.data_as(ctypes.c_void_p), it, best_len,
                               None if bt is None else bt.ctypes.data_as(ctypes.c_void_p)),
               "aco_restore")

    @property
    def iteration(self) -> int:
        v = ctypes.c_uint32()
        _check(lib.aco_get_iter(self._ctx, ctypes.byref(v)), "aco_get_iter")
        return int(v.value)

    def sync(self):
        _check(lib.aco_sync(self._ctx), "aco_sync")

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(512)
        _check(lib.aco_describe(self._ctx, buf, 512), "aco_describe")
        return buf.value.decode()

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib.aco_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def test_select(rows, feasible, u, tile: int = 8, waves: int = 1, stream=None):
    """R64 roulette on independent rows through the construction kernel's code
    of the given shape (tile cities per lane, waves wavefronts per ant).
    rows: (count, n) float32 torch tensor on the GPU; feasible: (count, n)
    uint8; u: (count,) float32.  Returns a (count,) int32 tensor."""
    import torch

    count, n = rows.shape
    ld = (n + 63) // 64 * 64
    padded = torch.zeros((count, ld), dtype=torch.float32, device=rows.device)
    padded[:, :n] = rows
    feas = feasible.to(torch.uint8).contiguous()
    uu = u.to(torch.float32).contiguous()
    out = torch.empty(count, dtype=torch.int32, device=rows.device)
    _check(lib.aco_test_select_shape(tile, waves, n, count, ctypes.c_void_p(padded.data_ptr()),
                                     ctypes.c_void_p(feas.data_ptr()),
                                     ctypes.c_void_p(uu.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
           "aco_test_select_shape")
    return out


def test_product_select(rows, feasible, u, stream=None):
    """Product-and-argmax selection on independent rows through the
    construction kernel's code.  rows, u: (count, n) float32 torch tensors on
    the GPU; feasible: (count, n) uint8.  Returns a (count,) int32 tensor."""
    import torch

    count, n = rows.shape
    ld = (n + 63) // 64 * 64
    padded = torch.zeros((count, ld), dtype=torch.float32, device=rows.device)
    padded[:, :n] = rows
    feas = feasible.to(torch.uint8).contiguous()
    uu = u.to(torch.float32).contiguous()
    out = torch.empty(count, dtype=torch.int32, device=rows.device)
    _check(lib.aco_test_product_select(n, count, ctypes.c_void_p(padded.data_ptr()),
                                       ctypes.c_void_p(feas.data_ptr()),
                                       ctypes.c_void_p(uu.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)),
           "aco_test_product_select")
    return out


def set_tile(n_lo: int, n_hi: int, cities_per_lane: int):
    _check(lib.aco_set_tile(n_lo, n_hi, cities_per_lane), "aco_set_tile")


def set_shape(n_lo: int, n_hi: int, cities_per_lane: int, waves_per_ant: int):
    """Construction shape for sizes n_lo..n_hi (aco_set_shape)."""
    _check(lib.aco_set_shape(n_lo, n_hi, cities_per_lane, waves_per_ant), "aco_set_shape")


def get_waves(n: int) -> int:
    return int(lib.aco_get_waves(n))


# (cities per lane, wavefronts per ant) of the autotuner's ms columns
SHAPES = ((4, 1), (8, 1), (8, 2), (4, 2), (4, 4))


def reset_tiles():
    """Restores the library's default construction tiles (aco_reset_tiles)."""
    lib.aco_reset_tiles()


def get_tile(n: int) -> int:
    return int(lib.aco_get_tile(n))


def autotune(sizes, reps: int = 3, device="cuda", stream=None):
    """Times every construction shape on synthetic instances of the given
    sizes (m = n) and sets the shape table; returns (chosen_tile,
    chosen_waves, ms) with ms of shape (len(sizes), len(SHAPES)), -1 where a
    shape does not support the size."""
    import torch

    sizes = np.ascontiguousarray(sorted(int(x) for x in sizes), np.int32)
    k = len(sizes)
    nbytes = workspace_bytes(int(sizes[-1]), int(sizes[-1]), atomic=False)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    tiles = np.zeros(k, np.int32)
    waves = np.zeros(k, np.int32)
    ms = np.zeros((k, len(SHAPES)), np.float32)
    _check(lib.aco_autotune(ctypes.c_void_p(ws.data_ptr()), nbytes,
                            sizes.ctypes.data_as(ctypes.c_void_p), k, reps,
                            _stream_handle(stream), tiles.ctypes.data_as(ctypes.c_void_p),
                            waves.ctypes.data_as(ctypes.c_void_p),
                            ms.ctypes.data_as(ctypes.c_void_p)), "aco_autotune")
    return tiles, waves, ms


class Batch:
    """Many independent instances resident on one GPU, advanced together.

    dists: list of (n_q, n_q) int32 matrices; params: list of dicts with keys
    m, alpha, beta, rho, seed (n comes from the matrix).  All launches go to
    `stream` (default: a new non-default torch stream, needed for graphs).
    """

    def __init__(self, dists, params, device="cuda", stream=None):
        import torch

        self.count = len(dists)
        self._dists = [as_dist(d) for d in dists]
        arr = (Params * self.count)()
        for q, (d, p) in enumerate(zip(self._dists, params)):
            arr[q] = Params(d.shape[0], p["m"], p.get("alpha", 1), p.get("beta", 2),
                            p.get("rho", 0.5), p.get("seed", 1))
        self.params = arr
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        nbytes = lib.aco_batch_workspace_bytes(self.count, arr)
        if nbytes == 0:
            _check(ACO_ERR_INVALID, "aco_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.workspace.record_stream(self.stream)
        ptrs = (ctypes.c_void_p * self.count)(*[d.ctypes.data for d in self._dists])
        self._b = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.aco_batch_init(ctypes.byref(self._b), self.count, arr, ptrs,
                                      ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                      _stream_handle(self.stream)), "aco_batch_init")

    def run(self, iters: int, graph: bool = True):
        _check(lib.aco_batch_run(self._b, iters, 1 if graph else 0), "aco_batch_run")

    def sync(self):
        _check(lib.aco_batch_sync(self._b), "aco_batch_sync")

    @property
    def config(self) -> dict:
        cfg = BatchConfig()
        _check(lib.aco_batch_get_config(self._b, ctypes.byref(cfg)), "aco_batch_get_config")
        return {"wg_per_cu": int(cfg.wg_per_cu), "tile4_max_n": int(cfg.tile4_max_n)}

    def set_config(self, wg_per_cu: int, tile4_max_n: int = -1):
        cfg = BatchConfig(wg_per_cu, tile4_max_n)
        _check(lib.aco_batch_set_config(self._b, ctypes.byref(cfg)), "aco_batch_set_config")

    def autotune(self, candidates, iters: int = 2):
        """candidates: (wg_per_cu, tile4_max_n) pairs.  Times each on this
        batch (advancing it, see aco_batch_autotune) and keeps the fastest;
        returns (best index, ms per iteration of every candidate)."""
        arr = (BatchConfig * len(candidates))(*[BatchConfig(w, t) for w, t in candidates])
        best = ctypes.c_int32(-1)
        ms = np.zeros(len(candidates), np.float32)
        _check(lib.aco_batch_autotune(self._b, arr, len(candidates), iters, ctypes.byref(best),
                                      ms.ctypes.data_as(ctypes.c_void_p)), "aco_batch_autotune")
        return int(best.value), ms

    def best(self, q: int):
        n = self._dists[q].shape[0]
        tour = np.empty(n + 1, np.uint16)
        length = ctypes.c_int64()
        _check(lib.aco_batch_read_best(self._b, q, tour.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.byref(length)), "aco_batch_read_best")
        return tour, int(length.value)

    def tours(self, q: int):
        n = self._dists[q].shape[0]
        m = self.params[q].m
        t = np.empty((m, n + 1), np.uint16)
        ln = np.empty(m, np.int64)
        _check(lib.aco_batch_read_tours(self._b, q, t.ctypes.data_as(ctypes.c_void_p),
                                        ln.ctypes.data_as(ctypes.c_void_p)),
               "aco_batch_read_tours")
        return t, ln

    def tau(self, q: int):
        n = self._dists[q].shape[0]
        out = np.empty((n, n), np.float32)
        _check(lib.aco_batch_read_tau(self._b, q, out.ctypes.data_as(ctypes.c_void_p)),
               "aco_batch_read_tau")
        return out

    def iteration(self, q: int) -> int:
        v = ctypes.c_uint32()
        _check(lib.aco_batch_get_iter(self._b, q, ctypes.byref(v)), "aco_batch_get_iter")
        return int(v.value)

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            lib.aco_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_copy(dst, src, stream=None):
    _check(lib.aco_probe_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                              src.numel() * src.element_size(), _stream_handle(stream)),
           "aco_probe_copy")


def probe_rows(mat, rows: int, ld: int, row_len: int, waves: int, steps: int, sink,
               stream=None, rows_in_flight: int = 1):
    _check(lib.aco_probe_rows_shape(ctypes.c_void_p(mat.data_ptr()), rows, ld, row_len, waves,
                                    steps, rows_in_flight, ctypes.c_void_p(sink.data_ptr()),
                                    _stream_handle(stream)), "aco_probe_rows_shape")


def probe_philox(waves: int, steps: int, seed: int, sink, stream=None):
    """sink: int32/uint32 torch tensor of waves * 64 elements on the GPU."""
    assert sink.numel() >= waves * 64
    _check(lib.aco_probe_philox(waves, steps, seed, ctypes.c_void_p(sink.data_ptr()),
                                _stream_handle(stream)), "aco_probe_philox")


def probe_read(src, reps: int, sink, stream=None, loads: int = 4, nontemporal: bool = False):
    _check(lib.aco_probe_read_shape(ctypes.c_void_p(src.data_ptr()),
                                    src.numel() * src.element_size(), reps, loads,
                                    1 if nontemporal else 0, ctypes.c_void_p(sink.data_ptr()),
                                    _stream_handle(stream)), "aco_probe_read_shape")
