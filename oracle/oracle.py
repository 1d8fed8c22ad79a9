"""Python side of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU baseline leg import
this module.  It marshals numpy arrays into the plain C oracle in
``oracle.c`` (built here with gcc) and adds a brute-force form for tiny
inputs written with Python loops straight from the definitions:

* embeddings: every injective tuple of data vertices is tested against the
  subgraph-isomorphism conditions (Section 2.1.4);
* maximum independent set (Section 2.4.2) by exhaustive search;
* MNI (Section 2.4.4) from the list of images;
* the greedy maximal independent set (Section 2.4.3) in lexicographic
  order of the tuples.

It shares no code with the HIP library.
"""

from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compiles oracle.c into liboracle.so with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _OgGraph(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("vlabel", ctypes.c_void_p), ("elabel", ctypes.c_void_p), ("directed", ctypes.c_int32)]


class _OgPattern(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("vlabel", ctypes.c_void_p),
                ("edges", ctypes.c_void_p), ("elabel", ctypes.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.og_tau.restype = ctypes.c_int64
        lib.og_tau.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_int32]
        lib.og_enumerate.restype = ctypes.c_int64
        lib.og_enumerate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        lib.og_support_literal.restype = ctypes.c_int64
        lib.og_support_literal.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_int64]
        lib.og_support_stream.restype = ctypes.c_int64
        lib.og_support_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_int64]
        lib.og_count.restype = ctypes.c_int
        lib.og_count.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p]
        lib.og_mni.restype = ctypes.c_int64
        lib.og_mni.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.og_greedy_rows.restype = ctypes.c_int64
        lib.og_greedy_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_void_p]
        lib.og_tuple_hash.restype = ctypes.c_uint64
        lib.og_tuple_hash.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64]
        lib.og_rows_digest.restype = None
        lib.og_rows_digest.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]
        lib.og_check_pattern.restype = ctypes.c_int
        lib.og_check_pattern.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class OracleGraph:
    """Holds the arrays alive for the C structs.  directed: row u lists the
    heads of the edges u -> v (Section 2.2's directed graphs)."""

    def __init__(self, row_ptr, col, vlabel, elabel=None, directed=False):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.vlabel = np.ascontiguousarray(vlabel, dtype=np.int32)
        self.elabel = (np.zeros(self.col.shape[0], dtype=np.int32) if elabel is None
                       else np.ascontiguousarray(elabel, dtype=np.int32))
        self.nv = self.row_ptr.shape[0] - 1
        self.directed = bool(directed)
        self.c = _OgGraph(self.nv, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.vlabel), _ptr(self.elabel),
                          1 if directed else 0)

    @classmethod
    def of(cls, g) -> "OracleGraph":
        return cls(g.row_ptr, g.col, g.vlabel, g.elabel, getattr(g, "directed", False))


class OraclePattern:
    def __init__(self, vlabel: Sequence[int], edges: Sequence[Tuple[int, int]],
                 elabel: Optional[Sequence[int]] = None):
        self.vlabel = np.ascontiguousarray(vlabel, dtype=np.int32)
        self.edges = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1), dtype=np.int32)
        m = self.edges.shape[0] // 2
        self.elabel = (np.zeros(m, dtype=np.int32) if elabel is None
                       else np.ascontiguousarray(elabel, dtype=np.int32))
        self.n = int(self.vlabel.shape[0])
        self.m = m
        self.c = _OgPattern(self.n, m, _ptr(self.vlabel), _ptr(self.edges), _ptr(self.elabel))

    @classmethod
    def of(cls, p) -> "OraclePattern":
        return cls(p.vlabel, p.edges, p.elabel)


def _as_graph(g) -> OracleGraph:
    return g if isinstance(g, OracleGraph) else OracleGraph.of(g)


def _as_pattern(p) -> OraclePattern:
    return p if isinstance(p, OraclePattern) else OraclePattern.of(p)


# ---------------------------------------------------------------------------
# thin wrappers
# ---------------------------------------------------------------------------

def tau(sigma: int, lam: float, n: int) -> int:
    """Threshold of the tau equation (Section 3.1.1), lambda in ppm."""
    return int(_load().og_tau(int(sigma), float(lam), int(n)))


def tau_eff(sigma: int, lam: float, n: int) -> int:
    """A pattern without embeddings is never frequent: the threshold is at least 1."""
    return max(tau(sigma, lam, n), 1)


def enumerate_embeddings(g, p, cap: int = 1 << 22) -> Tuple[int, np.ndarray]:
    """All embeddings in lexicographic order (first `cap` rows) and |M|."""
    G, P = _as_graph(g), _as_pattern(p)
    out = np.zeros((max(cap, 1), P.n), dtype=np.int32)
    cnt = _load().og_enumerate(ctypes.byref(G.c), ctypes.byref(P.c), _ptr(out), cap)
    if cnt < 0:
        raise ValueError("bad pattern")
    return int(cnt), out[:min(cnt, cap)]


def support_literal(g, p, cap: int = 1 << 22) -> Tuple[int, np.ndarray]:
    G, P = _as_graph(g), _as_pattern(p)
    sel = np.zeros((max(G.nv // max(P.n, 1) + 1, 1), P.n), dtype=np.int32)
    k = _load().og_support_literal(ctypes.byref(G.c), ctypes.byref(P.c), cap, _ptr(sel), sel.shape[0])
    if k == -2:
        raise OverflowError("embedding list does not fit")
    if k < 0:
        raise ValueError("bad pattern")
    return int(k), sel[:k]


def support_stream(g, p, stop_at: int = 0) -> Tuple[int, np.ndarray]:
    G, P = _as_graph(g), _as_pattern(p)
    sel = np.zeros((max(G.nv // max(P.n, 1) + 1, 1), P.n), dtype=np.int32)
    k = _load().og_support_stream(ctypes.byref(G.c), ctypes.byref(P.c), stop_at, _ptr(sel), sel.shape[0])
    if k < 0:
        raise ValueError("bad pattern")
    return int(k), sel[:k]


def count(g, p, cap: int) -> Tuple[int, bool, Tuple[int, int]]:
    G, P = _as_graph(g), _as_pattern(p)
    c = ctypes.c_int64(0)
    s = ctypes.c_int32(0)
    d = (ctypes.c_uint64 * 2)()
    rc = _load().og_count(ctypes.byref(G.c), ctypes.byref(P.c), cap, ctypes.byref(c), ctypes.byref(s), d)
    if rc != 0:
        raise ValueError("bad pattern")
    return int(c.value), bool(s.value), (int(d[0]), int(d[1]))


def mni(g, p) -> int:
    G, P = _as_graph(g), _as_pattern(p)
    return int(_load().og_mni(ctypes.byref(G.c), ctypes.byref(P.c)))


def tuple_hash(e: Sequence[int], seed: int) -> int:
    a = np.ascontiguousarray(e, dtype=np.int32)
    return int(_load().og_tuple_hash(_ptr(a), a.shape[0], seed))


def rows_digest(rows: np.ndarray, n: int) -> Tuple[int, int]:
    """(sum, xor) of the tuple hashes of the rows: the embedding digest's
    hash applied to any list of tuples, e.g. the selected set S."""
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1, n) if n else
                                np.zeros((0, 0), np.int32), dtype=np.int32)
    d = (ctypes.c_uint64 * 2)()
    _load().og_rows_digest(_ptr(rows) if rows.size else None, rows.shape[0], n, d)
    return int(d[0]), int(d[1])


def greedy_rows(rows: np.ndarray, nv: int) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    sel = np.zeros(max(rows.shape[0], 1), dtype=np.int64)
    k = _load().og_greedy_rows(_ptr(rows), rows.shape[0], rows.shape[1] if rows.ndim == 2 else 0, nv, _ptr(sel))
    return sel[:k]


def pattern_valid(p) -> bool:
    P = _as_pattern(p)
    return _load().og_check_pattern(ctypes.byref(P.c)) == 0


FULL = 0
VERDICT = 1


def query(g, p, sigma: int, lam: float, mode: int = FULL, count_cap: int = 1 << 62) -> Dict:
    """The full per-pattern result the device path must reproduce.

    FULL: exact support, verdict, tau, min(|M|, cap), saturation flag,
    digest, the selected embeddings in rank order and their digest
    (``sel_digest``: the same tuple hash over S).  VERDICT: the verdict
    only, with support = tau if frequent, else -1, and count = -1 (the
    search may stop once tau selections exist, Section 3.1.1).
    """
    P = _as_pattern(p)
    t = tau(sigma, lam, P.n)
    te = max(t, 1)
    if mode == VERDICT:
        k, _ = support_stream(g, P, stop_at=te)
        freq = k >= te
        return dict(tau=t, support=(t if freq else -1), frequent=int(freq), embedding_count=-1,
                    count_saturated=0, digest=(0, 0), selected=None, sel_digest=(0, 0))
    k, sel = support_stream(g, P)
    c, sat, dg = count(g, P, count_cap)
    return dict(tau=t, support=k, frequent=int(k >= te), embedding_count=c, count_saturated=int(sat),
                digest=(dg if not sat else (0, 0)), selected=sel, sel_digest=rows_digest(sel, P.n))


# ---------------------------------------------------------------------------
# Brute force for tiny inputs (pure Python, straight from the definitions)
# ---------------------------------------------------------------------------

def _adj_dict(g) -> Dict[Tuple[int, int], int]:
    G = _as_graph(g)
    d = {}
    for u in range(G.nv):
        for k in range(int(G.row_ptr[u]), int(G.row_ptr[u + 1])):
            d[(u, int(G.col[k]))] = int(G.elabel[k])
    return d


def brute_embeddings(g, p) -> List[Tuple[int, ...]]:
    """Every injective tuple satisfying Section 2.1.4, in lexicographic order
    (for a directed graph the rows hold out-edges only, so a pattern edge
    (a, b) needs the data edge f(a) -> f(b))."""
    G, P = _as_graph(g), _as_pattern(p)
    adj = _adj_dict(G)
    edges = [(int(P.edges[2 * k]), int(P.edges[2 * k + 1]), int(P.elabel[k])) for k in range(P.m)]
    out = []
    for t in itertools.permutations(range(G.nv), P.n):  # injective by construction, lexicographic
        if any(int(G.vlabel[t[i]]) != int(P.vlabel[i]) for i in range(P.n)):
            continue
        if all(adj.get((t[a], t[b])) == lab for a, b, lab in edges):
            out.append(tuple(t))
    return out


def brute_greedy(embs: List[Tuple[int, ...]]) -> List[Tuple[int, ...]]:
    used, sel = set(), []
    for e in embs:
        if used.isdisjoint(e):
            sel.append(e)
            used.update(e)
    return sel


def brute_mis(embs: List[Tuple[int, ...]]) -> int:
    """Maximum independent set size (Section 2.4.2) by exhaustive search over
    the distinct vertex sets (mappings with equal vertex sets are
    interchangeable for independence)."""
    sets = sorted({frozenset(e) for e in embs}, key=lambda s: sorted(s))
    best = 0

    def rec(i, used, size):
        nonlocal best
        if size + (len(sets) - i) <= best:
            return
        if i == len(sets):
            best = max(best, size)
            return
        if used.isdisjoint(sets[i]):
            rec(i + 1, used | sets[i], size + 1)
        rec(i + 1, used, size)

    rec(0, frozenset(), 0)
    return best


def brute_mni(embs: List[Tuple[int, ...]], n: int) -> int:
    if not embs:
        return 0
    return min(len({e[j] for e in embs}) for j in range(n))


def is_maximal_independent(sel: List[Tuple[int, ...]], embs: List[Tuple[int, ...]]) -> bool:
    used = set()
    for e in sel:
        if not used.isdisjoint(e):
            return False
        used.update(e)
    return all(not used.isdisjoint(e) for e in embs)
