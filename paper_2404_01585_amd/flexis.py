"""Python binding of the C ABI in include/flexis.h (argument marshalling only).

Every step of the support computation runs in the HIP library
``libflexis.so``; this module only converts numpy arrays / torch tensors and
patterns into the C structs and back.  PyTorch is used for the HIP stream
(``torch.cuda.current_stream()``) and, optionally, device-resident input
arrays.  If the library is not built, importing works but every call raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libflexis.so")

FX_OK = 0
FX_EINVAL = -1
FX_EGRAPH = -2
FX_EPATTERN = -3
FX_ENOMEM = -4
FX_EDEVICE = -5
FX_EBUSY = -6
FX_ETIMEOUT = -7
FX_ELIMIT = -8

MODE_FULL = 0
MODE_VERDICT = 1
MODE_MNI = 2  # minimum-image support (Section 2.4.4) instead of the greedy
MODE_MIS = 3  # exact maximum independent set (Section 2.4.2), small instances

_STATUS_NAMES = {0: "FX_OK", -1: "FX_EINVAL", -2: "FX_EGRAPH", -3: "FX_EPATTERN", -4: "FX_ENOMEM",
                 -5: "FX_EDEVICE", -6: "FX_EBUSY", -7: "FX_ETIMEOUT", -8: "FX_ELIMIT"}

# Every symbol include/flexis.h declares.
EXPORTS = ["fx_ctx_create", "fx_ctx_destroy", "fx_graph_load", "fx_graph_destroy", "fx_tau", "fx_support",
           "fx_enumerate", "fx_support_batch", "fx_ctx_stats", "fx_ctx_set", "fx_ctx_get", "fx_server_create",
           "fx_server_submit", "fx_server_poll", "fx_server_wait", "fx_server_stats", "fx_server_destroy",
           "fx_autotune", "fx_support_noalloc", "fx_alloc_calls", "fx_last_error", "fx_version"]

# fx_result.exit
EXIT_END = 0
EXIT_REACHED = 1
EXIT_BOUND = 2
EXIT_STATIC = 3
EXIT_EMPTY = 4

CTX_KERNEL_TIMING = 1
CTX_NO_DIGEST = 2


class FxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class CtxOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("hip_stream", ctypes.c_void_p), ("slice_rows", ctypes.c_int64),
                ("count_cap", ctypes.c_int64), ("mem_budget_bytes", ctypes.c_int64),
                ("run_index_bytes", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class GraphDesc(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_int64), ("num_adj", ctypes.c_int64), ("offset_bytes", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("vlabel", ctypes.c_void_p),
                ("elabel", ctypes.c_void_p), ("on_device", ctypes.c_int32), ("directed", ctypes.c_int32)]


class PatternC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("vlabel", ctypes.c_void_p),
                ("edges", ctypes.c_void_p), ("elabel", ctypes.c_void_p)]


class ServerOptsC(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("slice_rows", ctypes.c_int64), ("mem_budget_bytes", ctypes.c_int64),
                ("step_candidates", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class TuneC(ctypes.Structure):
    _fields_ = [("slice_rows", ctypes.c_int64), ("step_candidates", ctypes.c_int64),
                ("items_per_thread", ctypes.c_int32), ("last_span_init", ctypes.c_int32), ("best_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double), ("trials", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("max_active", ctypes.c_int32)]

    def to_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class StatsC(ctypes.Structure):
    _fields_ = [("probe_launches", ctypes.c_uint64), ("probe_ms", ctypes.c_double),
                ("probe_alg_bytes", ctypes.c_uint64), ("scatter_launches", ctypes.c_uint64),
                ("scatter_ms", ctypes.c_double), ("scatter_alg_bytes", ctypes.c_uint64),
                ("greedy_launches", ctypes.c_uint64), ("greedy_ms", ctypes.c_double), ("steps", ctypes.c_uint64),
                ("syncs", ctypes.c_uint64), ("queries", ctypes.c_uint64), ("reoffered", ctypes.c_uint64),
                ("promotions", ctypes.c_uint64), ("host_ms", ctypes.c_double), ("wait_ms", ctypes.c_double),
                ("exits_reached", ctypes.c_uint64), ("exits_bound", ctypes.c_uint64),
                ("lone_promotions", ctypes.c_uint64), ("probe_ref_bytes", ctypes.c_uint64),
                ("scatter_ref_bytes", ctypes.c_uint64), ("greedy_ref_bytes", ctypes.c_uint64),
                ("probed", ctypes.c_uint64), ("probe_ref_row_bytes", ctypes.c_uint64),
                ("chains", ctypes.c_uint64), ("chain_steps", ctypes.c_uint64)]

    def to_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ResultC(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_int64), ("support", ctypes.c_int64), ("frequent", ctypes.c_int32),
                ("count_saturated", ctypes.c_int32), ("embedding_count", ctypes.c_int64),
                ("digest", ctypes.c_uint64 * 2), ("steps", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("device_ms", ctypes.c_double), ("alg_bytes", ctypes.c_uint64), ("sel_digest", ctypes.c_uint64 * 2),
                ("status", ctypes.c_int32), ("exit", ctypes.c_int32)]

    def to_dict(self) -> Dict:
        return dict(tau=self.tau, support=self.support, frequent=self.frequent,
                    count_saturated=self.count_saturated, embedding_count=self.embedding_count,
                    digest=(int(self.digest[0]), int(self.digest[1])), steps=self.steps, rounds=self.rounds,
                    device_ms=self.device_ms, alg_bytes=int(self.alg_bytes),
                    sel_digest=(int(self.sel_digest[0]), int(self.sel_digest[1])), status=self.status,
                    exit=self.exit)


# numpy views of the C structs (same field order, offsets and sizes)
PATTERN_DTYPE = np.dtype([("n", "<i4"), ("m", "<i4"), ("vlabel", "<u8"), ("edges", "<u8"), ("elabel", "<u8")])
RESULT_DTYPE = np.dtype([("tau", "<i8"), ("support", "<i8"), ("frequent", "<i4"), ("count_saturated", "<i4"),
                         ("embedding_count", "<i8"), ("digest", "<u8", (2,)), ("steps", "<i4"), ("rounds", "<i4"),
                         ("device_ms", "<f8"), ("alg_bytes", "<u8"), ("sel_digest", "<u8", (2,)), ("status", "<i4"),
                         ("exit", "<i4")])
assert PATTERN_DTYPE.itemsize == ctypes.sizeof(PatternC)
assert RESULT_DTYPE.itemsize == ctypes.sizeof(ResultC)


class PatternBatch:
    """A list of patterns packed once into fx_pattern structs (for repeated batches)."""

    def __init__(self, patterns):
        self.patterns = list(patterns)
        k = len(self.patterns)
        n = np.array([len(p.vlabel) for p in self.patterns], dtype=np.int64)
        m = np.array([len(p.edges) for p in self.patterns], dtype=np.int64)
        self.vl = np.ascontiguousarray(np.concatenate([np.asarray(p.vlabel, dtype=np.int32) for p in self.patterns])
                                       if k else np.zeros(1, np.int32), dtype=np.int32)
        self.ed = np.ascontiguousarray(np.concatenate([np.asarray(p.edges, dtype=np.int32).reshape(-1)
                                                       for p in self.patterns]) if k else np.zeros(1, np.int32),
                                       dtype=np.int32)
        self.el = np.ascontiguousarray(np.concatenate([np.asarray(p.elabel, dtype=np.int32) for p in self.patterns])
                                       if k else np.zeros(1, np.int32), dtype=np.int32)
        if self.ed.size == 0:
            self.ed = np.zeros(1, np.int32)
        if self.el.size == 0:
            self.el = np.zeros(1, np.int32)
        vo = np.concatenate([[0], np.cumsum(n)[:-1]]) if k else np.zeros(0, np.int64)
        eo = np.concatenate([[0], np.cumsum(m)[:-1]]) if k else np.zeros(0, np.int64)
        self.arr = np.zeros(max(k, 1), dtype=PATTERN_DTYPE)
        self.arr["n"][:k] = n
        self.arr["m"][:k] = m
        self.arr["vlabel"][:k] = self.vl.ctypes.data + 4 * vo
        self.arr["edges"][:k] = self.ed.ctypes.data + 8 * eo
        self.arr["elabel"][:k] = self.el.ctypes.data + 4 * eo

    def __len__(self):
        return len(self.patterns)


_lib = None


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Loads libflexis.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run paper_2404_01585_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.fx_last_error.restype = ctypes.c_char_p
    lib.fx_last_error.argtypes = []
    lib.fx_version.restype = ctypes.c_char_p
    lib.fx_version.argtypes = []
    lib.fx_tau.restype = ctypes.c_int32
    lib.fx_tau.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int32, P]
    lib.fx_ctx_create.restype = ctypes.c_int32
    lib.fx_ctx_create.argtypes = [P, P]
    lib.fx_ctx_destroy.restype = ctypes.c_int32
    lib.fx_ctx_destroy.argtypes = [P]
    lib.fx_graph_load.restype = ctypes.c_int32
    lib.fx_graph_load.argtypes = [P, P, P]
    lib.fx_graph_destroy.restype = ctypes.c_int32
    lib.fx_graph_destroy.argtypes = [P]
    lib.fx_support.restype = ctypes.c_int32
    lib.fx_support.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, P, P, ctypes.c_int64]
    lib.fx_enumerate.restype = ctypes.c_int32
    lib.fx_enumerate.argtypes = [P, P, P, ctypes.c_int64, P]
    lib.fx_server_create.restype = ctypes.c_int32
    lib.fx_server_create.argtypes = [P, P, P]
    lib.fx_server_submit.restype = ctypes.c_int32
    lib.fx_server_submit.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, P]
    lib.fx_server_poll.restype = ctypes.c_int32
    lib.fx_server_poll.argtypes = [P, ctypes.c_uint64, P, P]
    lib.fx_server_wait.restype = ctypes.c_int32
    lib.fx_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.c_int64, P]
    lib.fx_server_stats.restype = ctypes.c_int32
    lib.fx_server_stats.argtypes = [P, P]
    lib.fx_server_destroy.restype = ctypes.c_int32
    lib.fx_server_destroy.argtypes = [P]
    lib.fx_autotune.restype = ctypes.c_int32
    lib.fx_autotune.argtypes = [P, ctypes.c_int32, P, P, P, ctypes.c_int32, ctypes.c_char_p, P]
    lib.fx_ctx_stats.restype = ctypes.c_int32
    lib.fx_ctx_stats.argtypes = [P, P, ctypes.c_int32]
    lib.fx_ctx_set.restype = ctypes.c_int32
    lib.fx_ctx_set.argtypes = [P, ctypes.c_char_p, ctypes.c_int64]
    lib.fx_ctx_get.restype = ctypes.c_int32
    lib.fx_ctx_get.argtypes = [P, ctypes.c_char_p, P]
    lib.fx_support_noalloc.restype = ctypes.c_int32
    lib.fx_support_noalloc.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, P]
    lib.fx_alloc_calls.restype = ctypes.c_uint64
    lib.fx_alloc_calls.argtypes = []
    lib.fx_support_batch.restype = ctypes.c_int32
    lib.fx_support_batch.argtypes = [P, ctypes.c_int32, P, P, P, ctypes.c_int32, P]
    _lib = lib
    return lib


def _check(status: int):
    if status != FX_OK:
        raise FxError(status, load_library().fx_last_error().decode(errors="replace"))


def alloc_calls() -> int:
    """fx_alloc_calls: device and pinned-host allocations made by the library so far."""
    return int(load_library().fx_alloc_calls())


def last_error() -> str:
    return load_library().fx_last_error().decode(errors="replace")


def tau(sigma: int, lam: float, n: int) -> int:
    out = ctypes.c_int64(0)
    _check(load_library().fx_tau(int(sigma), float(lam), int(n), ctypes.byref(out)))
    return int(out.value)


class _PatternHolder:
    """Keeps the numpy arrays of a pattern alive while C holds pointers to them."""

    def __init__(self, vlabel: Sequence[int], edges: Sequence[Tuple[int, int]], elabel: Optional[Sequence[int]]):
        self.vl = np.ascontiguousarray(vlabel, dtype=np.int32)
        self.ed = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1), dtype=np.int32)
        m = self.ed.shape[0] // 2
        self.el = (np.zeros(m, dtype=np.int32) if elabel is None
                   else np.ascontiguousarray(elabel, dtype=np.int32))
        self.c = PatternC(self.vl.shape[0], m, self.vl.ctypes.data, self.ed.ctypes.data if m else None,
                          self.el.ctypes.data if m else None)

    @classmethod
    def of(cls, p) -> "_PatternHolder":
        return cls(p.vlabel, p.edges, p.elabel)


def _current_stream() -> int:
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


class Context:
    """fx_ctx: a device, a stream, and the workspace sizing."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, slice_rows: int = 0, count_cap: int = 0,
                 kernel_timing: bool = False, mem_budget_bytes: int = 0, no_digest: bool = False,
                 run_index_bytes: int = 0):
        lib = load_library()
        if stream is None:
            import torch
            torch.cuda.set_device(device)
            stream = _current_stream()
        self.stream = stream
        self._opts = CtxOpts(device, stream or None, slice_rows, count_cap, mem_budget_bytes, run_index_bytes,
                             (CTX_KERNEL_TIMING if kernel_timing else 0) | (CTX_NO_DIGEST if no_digest else 0))
        self._h = ctypes.c_void_p()
        _check(lib.fx_ctx_create(ctypes.byref(self._opts), ctypes.byref(self._h)))
        self.count_cap = count_cap if count_cap > 0 else (1 << 62)

    @property
    def handle(self):
        return self._h

    def stats(self, reset: bool = False) -> Dict:
        st = StatsC()
        _check(load_library().fx_ctx_stats(self._h, ctypes.byref(st), 1 if reset else 0))
        return st.to_dict()

    def set(self, key: str, value: int) -> None:
        """fx_ctx_set: an engine tunable by name (launch shape, scheduling)."""
        _check(load_library().fx_ctx_set(self._h, key.encode(), int(value)))

    def get(self, key: str) -> int:
        out = ctypes.c_int64(0)
        _check(load_library().fx_ctx_get(self._h, key.encode(), ctypes.byref(out)))
        return int(out.value)

    def load_graph(self, g, on_device: bool = False) -> "DeviceGraph":
        return DeviceGraph(self, g, on_device=on_device)

    def close(self):
        if self._h:
            _check(load_library().fx_ctx_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class DeviceGraph:
    """fx_graph: a data graph resident on the device."""

    def __init__(self, ctx: Context, g, on_device: bool = False):
        lib = load_library()
        self.ctx = ctx
        self.nv = int(g.row_ptr.shape[0] - 1)
        if on_device:
            import torch
            rp = g.row_ptr if isinstance(g.row_ptr, torch.Tensor) else torch.from_numpy(np.asarray(g.row_ptr))
            keep = [None if t is None else (t.contiguous() if t.is_cuda else t.contiguous().cuda())
                    for t in (rp, _t(g.col), _t(g.vlabel), _t(g.elabel))]
            self._keep = keep
            ob = keep[0].element_size()
            desc = GraphDesc(self.nv, int(keep[1].numel()), ob, keep[0].data_ptr(), keep[1].data_ptr(),
                             keep[2].data_ptr(), None if keep[3] is None else keep[3].data_ptr(), 1,
                             1 if getattr(g, "directed", False) else 0)
        else:
            rp = np.ascontiguousarray(g.row_ptr)
            if rp.dtype not in (np.int32, np.int64):
                rp = rp.astype(np.int64)
            col = np.ascontiguousarray(g.col, dtype=np.int32)
            vl = np.ascontiguousarray(g.vlabel, dtype=np.int32)
            el = None if g.elabel is None else np.ascontiguousarray(g.elabel, dtype=np.int32)
            self._keep = [rp, col, vl, el]
            desc = GraphDesc(self.nv, int(col.shape[0]), rp.dtype.itemsize, rp.ctypes.data,
                             col.ctypes.data if col.shape[0] else None, vl.ctypes.data,
                             el.ctypes.data if (el is not None and el.shape[0]) else None, 0,
                             1 if getattr(g, "directed", False) else 0)
        self._h = ctypes.c_void_p()
        _check(lib.fx_graph_load(ctx.handle, ctypes.byref(desc), ctypes.byref(self._h)))
        self._keep = None

    def support(self, p, sigma: int, lam: float, mode: int = MODE_FULL, selected_cap: int = 0) -> Dict:
        """fx_support for one pattern; returns the fx_result fields (+ 'selected')."""
        ph = _PatternHolder.of(p)
        res = ResultC()
        sel = np.zeros((max(selected_cap, 1), ph.vl.shape[0]), dtype=np.int32)
        _check(load_library().fx_support(self._h, ctypes.byref(ph.c), int(sigma), float(lam), int(mode),
                                         ctypes.byref(res), sel.ctypes.data if selected_cap else None,
                                         int(selected_cap)))
        d = res.to_dict()
        if selected_cap and mode == MODE_FULL:
            d["selected"] = sel[:min(selected_cap, max(res.support, 0))]
        return d

    def support_noalloc(self, p, sigma: int, lam: float, mode: int = MODE_FULL) -> Dict:
        """fx_support_noalloc: fx_support without any allocation (static scratch array)."""
        ph = _PatternHolder.of(p)
        res = ResultC()
        _check(load_library().fx_support_noalloc(self._h, ctypes.byref(ph.c), int(sigma), float(lam), int(mode),
                                                 ctypes.byref(res)))
        return res.to_dict()

    def enumerate(self, p, cap: int) -> Tuple[int, np.ndarray]:
        """fx_enumerate: |M| and the first `cap` embeddings in rank order."""
        ph = _PatternHolder.of(p)
        rows = np.zeros((max(cap, 1), ph.vl.shape[0]), dtype=np.int32)
        cnt = ctypes.c_int64(0)
        _check(load_library().fx_enumerate(self._h, ctypes.byref(ph.c), rows.ctypes.data if cap else None,
                                           int(cap), ctypes.byref(cnt)))
        return int(cnt.value), rows[:min(cap, cnt.value)]

    def support_batch_array(self, batch: "PatternBatch", sigma, lam, mode: int = MODE_FULL) -> np.ndarray:
        """fx_support_batch; results as a numpy array of RESULT_DTYPE."""
        k = len(batch)
        sg = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.int64), (k,)))
        lm = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (k,)))
        res = np.zeros(max(k, 1), dtype=RESULT_DTYPE)
        _check(load_library().fx_support_batch(self._h, k, batch.arr.ctypes.data, sg.ctypes.data, lm.ctypes.data,
                                               int(mode), res.ctypes.data))
        return res[:k]

    def autotune(self, batch: "PatternBatch", sigma, lam, mode: int = MODE_FULL,
                 cache_path: Optional[str] = None) -> Dict:
        """fx_autotune on a sample batch; the chosen setting stays in the context."""
        k = len(batch)
        sg = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.int64), (k,)))
        lm = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (k,)))
        r = TuneC()
        _check(load_library().fx_autotune(self._h, k, batch.arr.ctypes.data, sg.ctypes.data, lm.ctypes.data,
                                          int(mode), cache_path.encode() if cache_path else None, ctypes.byref(r)))
        return r.to_dict()

    def support_batch(self, patterns: List, sigma: Sequence[int], lam: Sequence[float],
                      mode: int = MODE_FULL) -> List[Dict]:
        res = self.support_batch_array(PatternBatch(patterns), sigma, lam, mode)
        out = []
        for r in res:
            d = {k: (int(r[k]) if k != "device_ms" else float(r[k])) for k in RESULT_DTYPE.names
                 if k not in ("digest", "sel_digest")}
            d["digest"] = (int(r["digest"][0]), int(r["digest"][1]))
            d["sel_digest"] = (int(r["sel_digest"][0]), int(r["sel_digest"][1]))
            out.append(d)
        return out

    def close(self):
        if self._h:
            _check(load_library().fx_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Server:
    """fx_server: continuous-batching support queries over a resident graph.

    submit/poll/wait are thread-safe (ctypes releases the GIL during calls)."""

    def __init__(self, graph: "DeviceGraph", max_active: int = 0, slice_rows: int = 0, mem_budget_bytes: int = 0,
                 step_candidates: int = 0, no_digest: bool = False):
        self.graph = graph
        self._opts = ServerOptsC(max_active, slice_rows, mem_budget_bytes, step_candidates,
                                 CTX_NO_DIGEST if no_digest else 0)
        self._h = ctypes.c_void_p()
        _check(load_library().fx_server_create(graph._h, ctypes.byref(self._opts), ctypes.byref(self._h)))

    def submit(self, p, sigma: int, lam: float, mode: int = MODE_FULL) -> int:
        ph = _PatternHolder.of(p)
        t = ctypes.c_uint64(0)
        _check(load_library().fx_server_submit(self._h, ctypes.byref(ph.c), int(sigma), float(lam), int(mode),
                                               ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int) -> Optional[Dict]:
        res = ResultC()
        done = ctypes.c_int32(0)
        _check(load_library().fx_server_poll(self._h, ticket, ctypes.byref(res), ctypes.byref(done)))
        return res.to_dict() if done.value else None

    def wait(self, ticket: int, timeout_us: int = -1) -> Dict:
        res = ResultC()
        _check(load_library().fx_server_wait(self._h, ticket, int(timeout_us), ctypes.byref(res)))
        return res.to_dict()

    def stats(self) -> Dict:
        st = StatsC()
        _check(load_library().fx_server_stats(self._h, ctypes.byref(st)))
        return st.to_dict()

    def close(self):
        if self._h:
            _check(load_library().fx_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _t(a):
    import torch
    if a is None:
        return None
    return a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
