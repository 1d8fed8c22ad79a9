"""Seeded synthetic inputs: labeled data graphs and candidate patterns.

This module only draws inputs. It holds none of the support-counting
arithmetic and is shared by the oracle-side tests and the device path, so
that both see identical bytes for a given seed.

Graph shapes follow the paper's workloads (Section 4, Table 1: undirected
social / peer-to-peer graphs with a handful of random vertex and edge labels)
and the synthetic stand-ins used for them here:

* ``erdos_renyi``   uniform random pairs (the tiny 1K-vertex case);
* ``chung_lu``      power-law expected degrees with a structural cutoff;
* ``rmat``          recursive-matrix graph (scale 22 case).

Every generator returns a simple undirected graph: self-loops dropped,
duplicates removed, and sampling continues until exactly ``m`` unique edges
exist.  Vertex ids are then permuted by a seeded permutation and labels are
drawn i.i.d. (vertex labels uniform or Zipf, edge labels uniform per
undirected edge).  The result is a symmetric CSR whose rows are ascending.
"""

from __future__ import annotations

import dataclasses
from collections import deque
from typing import List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class Graph:
    """Symmetric CSR with vertex and edge labels (host numpy arrays); with
    directed=True row u lists the heads of the edges u -> v instead."""

    row_ptr: np.ndarray  # int32 or int64 [nv+1]
    col: np.ndarray  # int32 [2|E|] (directed: [|E|]), ascending per row
    vlabel: np.ndarray  # int32 [nv]
    elabel: np.ndarray  # int32 [2|E|], equal for (u,v) and (v,u) (directed: one per edge)
    name: str = ""
    directed: bool = False

    @property
    def num_vertices(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def num_adj(self) -> int:
        return int(self.col.shape[0])

    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]

    def edge_list(self) -> np.ndarray:
        """Undirected edges (u < v) with their labels, shape [|E|, 3]."""
        src = np.repeat(np.arange(self.num_vertices, dtype=np.int64), self.degree())
        dst = self.col.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep], self.elabel[keep].astype(np.int64)], axis=1)


@dataclasses.dataclass
class Pattern:
    """Connected labeled pattern; vertices numbered 0..n-1 as submitted."""

    vlabel: List[int]
    edges: List[Tuple[int, int]]
    elabel: List[int]

    @property
    def n(self) -> int:
        return len(self.vlabel)

    @property
    def m(self) -> int:
        return len(self.edges)


# ---------------------------------------------------------------------------
# CSR assembly
# ---------------------------------------------------------------------------

def csr_from_edges(nv: int, u: np.ndarray, v: np.ndarray, el: np.ndarray,
                   vlabel: np.ndarray, offset_dtype=np.int32, name: str = "") -> Graph:
    """Builds the symmetric CSR of unique undirected edges (u_i, v_i, el_i)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    el = np.asarray(el, dtype=np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    lab = np.concatenate([el, el])
    order = np.argsort(src * nv + dst)  # keys are unique: the (src, dst) order
    src, dst, lab = src[order], dst[order], lab[order]
    counts = np.bincount(src, minlength=nv)
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(row_ptr=row_ptr.astype(offset_dtype), col=dst.astype(np.int32),
                 vlabel=np.asarray(vlabel, dtype=np.int32), elabel=lab.astype(np.int32), name=name)


def csr_from_arcs(nv: int, u: np.ndarray, v: np.ndarray, el: np.ndarray, vlabel: np.ndarray,
                  offset_dtype=np.int64, name: str = "") -> Graph:
    """Builds the directed CSR (row u: heads of the arcs u -> v, ascending) of
    unique arcs (u_i, v_i, el_i)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    el = np.asarray(el, dtype=np.int64)
    order = np.argsort(u * nv + v)
    u, v, el = u[order], v[order], el[order]
    counts = np.bincount(u, minlength=nv)
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(row_ptr=row_ptr.astype(offset_dtype), col=v.astype(np.int32),
                 vlabel=np.asarray(vlabel, dtype=np.int32), elabel=el.astype(np.int32), name=name, directed=True)


def tiny_random_digraph(rng: np.random.Generator, nv: int, p: float, n_vlabels: int, n_elabels: int) -> Graph:
    """Directed G(n, p): each ordered pair an arc with probability p (both
    directions of a pair may occur, with their own labels), random labels."""
    ii, jj = np.nonzero(~np.eye(nv, dtype=bool))
    keep = rng.random(ii.shape[0]) < p
    u, v = ii[keep], jj[keep]
    el = rng.integers(0, n_elabels, size=u.shape[0]) if n_elabels > 1 else np.zeros(u.shape[0], dtype=np.int64)
    vl = rng.integers(0, n_vlabels, size=nv)
    return csr_from_arcs(nv, u, v, el, vl, name="tiny_directed")


def random_directed_pattern(rng: np.random.Generator, n: int, n_vlabels: int, n_elabels: int,
                            extra_edge_p: float = 0.3, reciprocal_p: float = 0.2,
                            prefix_connected: bool = True) -> Pattern:
    """A random weakly connected directed pattern: a random orientation of
    random_connected_pattern's edges, some made reciprocal (both directions,
    each with its own label)."""
    base = random_connected_pattern(rng, n, n_vlabels, n_elabels, extra_edge_p, prefix_connected)
    edges, labels = [], []
    for (a, b), l in zip(base.edges, base.elabel):
        if rng.random() < 0.5:
            a, b = b, a
        edges.append((a, b))
        labels.append(l)
        if rng.random() < reciprocal_p:
            edges.append((b, a))
            labels.append(int(rng.integers(0, n_elabels)) if n_elabels > 1 else 0)
    return Pattern(vlabel=base.vlabel, edges=edges, elabel=labels)


def _unique_edges(nv: int, draw, m: int, rng: np.random.Generator) -> Tuple[np.ndarray, np.ndarray]:
    """Keeps drawing endpoint batches until exactly m unique simple edges exist.

    ``draw(k)`` returns two int64 arrays of k endpoints.  Edges keep the order
    in which they were first drawn, so the first m unique ones are kept.
    """
    keys = np.empty(0, dtype=np.int64)
    need = m
    batch = int(m * 1.25) + 64
    while True:
        a, b = draw(batch)
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        ok = lo != hi
        k = lo[ok] * nv + hi[ok]
        keys = np.concatenate([keys, k])
        _, first = np.unique(keys, return_index=True)
        if first.shape[0] >= m:
            first.sort()
            keys = keys[first[:m]]
            break
        first.sort()
        keys = keys[first]
        need = m - keys.shape[0]
        batch = int(need * 1.5) + 64
    return keys // nv, keys % nv


def _permute_and_label(nv: int, u: np.ndarray, v: np.ndarray, rng: np.random.Generator,
                       n_vlabels: int, vlabel_zipf: Optional[float], n_elabels: int,
                       offset_dtype, name: str) -> Graph:
    perm = rng.permutation(nv).astype(np.int64)
    u = perm[u]
    v = perm[v]
    vlabel = draw_labels(rng, nv, n_vlabels, vlabel_zipf)
    el = rng.integers(0, n_elabels, size=u.shape[0], dtype=np.int64) if n_elabels > 1 \
        else np.zeros(u.shape[0], dtype=np.int64)
    return csr_from_edges(nv, u, v, el, vlabel, offset_dtype=offset_dtype, name=name)


def draw_labels(rng: np.random.Generator, count: int, n_labels: int,
                zipf_s: Optional[float]) -> np.ndarray:
    """I.i.d. labels in [0, n_labels): uniform, or P(k) proportional to (k+1)^-s."""
    if n_labels <= 1:
        return np.zeros(count, dtype=np.int32)
    if zipf_s is None:
        return rng.integers(0, n_labels, size=count).astype(np.int32)
    w = (np.arange(n_labels, dtype=np.float64) + 1.0) ** (-zipf_s)
    w /= w.sum()
    return rng.choice(n_labels, size=count, p=w).astype(np.int32)


# ---------------------------------------------------------------------------
# Graph families
# ---------------------------------------------------------------------------

def erdos_renyi(nv: int, m: int, seed: int, n_vlabels: int = 5, vlabel_zipf=None,
                n_elabels: int = 1, offset_dtype=np.int32) -> Graph:
    rng = np.random.default_rng(seed)

    def draw(k):
        return rng.integers(0, nv, size=k, dtype=np.int64), rng.integers(0, nv, size=k, dtype=np.int64)

    u, v = _unique_edges(nv, draw, m, rng)
    return _permute_and_label(nv, u, v, rng, n_vlabels, vlabel_zipf, n_elabels, offset_dtype,
                              f"er_{nv}_{m}_s{seed}")


def chung_lu_weights(nv: int, m: int, gamma: float) -> np.ndarray:
    """Expected degrees w_i ~ (i+1)^(-1/(gamma-1)), mean 2m/nv, capped at sqrt(2m)."""
    w = (np.arange(nv, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    cap = np.sqrt(2.0 * m)
    target = 2.0 * m
    for _ in range(64):
        w *= target / w.sum()
        over = w > cap
        if not over.any():
            break
        w[over] = cap
    return w


def chung_lu(nv: int, m: int, gamma: float, seed: int, n_vlabels: int, vlabel_zipf=None,
             n_elabels: int = 1, offset_dtype=np.int32) -> Graph:
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(nv, m, gamma)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(k):
        a = np.searchsorted(cdf, rng.random(k), side="right")
        b = np.searchsorted(cdf, rng.random(k), side="right")
        return np.minimum(a, nv - 1).astype(np.int64), np.minimum(b, nv - 1).astype(np.int64)

    u, v = _unique_edges(nv, draw, m, rng)
    return _permute_and_label(nv, u, v, rng, n_vlabels, vlabel_zipf, n_elabels, offset_dtype,
                              f"cl_{nv}_{m}_g{gamma}_s{seed}")


def rmat(scale: int, m: int, seed: int, abcd=(0.57, 0.19, 0.19, 0.05), n_vlabels: int = 50,
         vlabel_zipf=1.1, n_elabels: int = 4, offset_dtype=np.int64) -> Graph:
    rng = np.random.default_rng(seed)
    nv = 1 << scale
    a, b, c, _ = abcd
    t1, t2, t3 = a, a + b, a + b + c

    def draw(k):
        src = np.zeros(k, dtype=np.int64)
        dst = np.zeros(k, dtype=np.int64)
        for _lvl in range(scale):
            r = rng.random(k, dtype=np.float32)
            bit_dst = ((r >= t1) & (r < t2)) | (r >= t3)
            bit_src = r >= t2
            src = (src << 1) | bit_src
            dst = (dst << 1) | bit_dst
        return src, dst

    u, v = _unique_edges(nv, draw, m, rng)
    return _permute_and_label(nv, u, v, rng, n_vlabels, vlabel_zipf, n_elabels, offset_dtype,
                              f"rmat_{scale}_{m}_s{seed}")


def tiny_random_graph(rng: np.random.Generator, nv: int, p: float, n_vlabels: int,
                      n_elabels: int) -> Graph:
    """G(n, p) with random labels, for brute-force cross-checks on tiny inputs."""
    iu, ju = np.triu_indices(nv, k=1)
    keep = rng.random(iu.shape[0]) < p
    u, v = iu[keep], ju[keep]
    el = rng.integers(0, n_elabels, size=u.shape[0]) if n_elabels > 1 else np.zeros(u.shape[0], dtype=np.int64)
    vl = rng.integers(0, n_vlabels, size=nv)
    return csr_from_edges(nv, u, v, el, vl, name="tiny")


# ---------------------------------------------------------------------------
# The named workloads (synthetic stand-ins for the paper's datasets)
# ---------------------------------------------------------------------------

WORKLOADS = {
    # name: (builder, kwargs)
    "er1k": dict(kind="er", nv=1000, m=4000, seed=1, n_vlabels=5, vlabel_zipf=None, n_elabels=1),
    "cl100k": dict(kind="cl", nv=100_000, m=500_000, gamma=2.1, seed=2, n_vlabels=20, vlabel_zipf=1.2,
                   n_elabels=3),
    "cl1m": dict(kind="cl", nv=1_000_000, m=8_000_000, gamma=2.3, seed=3, n_vlabels=30, vlabel_zipf=1.0,
                 n_elabels=1),
    "rmat22": dict(kind="rmat", scale=22, m=40_000_000, seed=5, n_vlabels=50, vlabel_zipf=1.1, n_elabels=4),
}


def workload_graph(name: str) -> Graph:
    cfg = dict(WORKLOADS[name])
    kind = cfg.pop("kind")
    if kind == "er":
        return erdos_renyi(cfg["nv"], cfg["m"], cfg["seed"], cfg["n_vlabels"], cfg["vlabel_zipf"],
                           cfg["n_elabels"])
    if kind == "cl":
        return chung_lu(cfg["nv"], cfg["m"], cfg["gamma"], cfg["seed"], cfg["n_vlabels"], cfg["vlabel_zipf"],
                        cfg["n_elabels"])
    if kind == "rmat":
        return rmat(cfg["scale"], cfg["m"], cfg["seed"], n_vlabels=cfg["n_vlabels"],
                    vlabel_zipf=cfg["vlabel_zipf"], n_elabels=cfg["n_elabels"])
    raise KeyError(name)


# ---------------------------------------------------------------------------
# Pattern sampling (connected subgraphs of the data graph)
# ---------------------------------------------------------------------------

def _edge_label(g: Graph, u: int, v: int) -> int:
    nb = g.neighbors(u)
    k = int(np.searchsorted(nb, v))
    assert k < nb.shape[0] and nb[k] == v
    return int(g.elabel[int(g.row_ptr[u]) + k])


def _bfs_number(n: int, edges: List[Tuple[int, int]], start: int) -> List[int]:
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    order, seen = [], [False] * n
    dq = deque([start])
    seen[start] = True
    while dq:
        x = dq.popleft()
        order.append(x)
        for y in sorted(adj[x]):
            if not seen[y]:
                seen[y] = True
                dq.append(y)
    return order


def sample_pattern(g: Graph, rng: np.random.Generator, k: int, shape: str,
                   max_tries: int = 200) -> Optional[Pattern]:
    """Samples a connected k-vertex subgraph of g of the given shape.

    shape: "tree" (random spanning tree of a grown vertex set), "chord" (tree
    plus one random non-tree induced edge) or "cycle" (a random simple path
    whose ends are adjacent).  Labels come from g, so the pattern has at least
    one embedding.  Vertices are numbered in BFS order from the vertex with the
    rarest label, which makes every prefix connected.
    """
    if shape == "cycle" and k < 3:
        shape = "tree"  # a simple cycle needs three vertices
    nv = g.num_vertices
    deg = g.degree()
    vcount = np.bincount(g.vlabel, minlength=int(g.vlabel.max()) + 1)
    def rand_nb(x, excl):
        """A uniformly random neighbour of x outside excl, or None."""
        nb = g.neighbors(x)
        d = nb.shape[0]
        if d == 0:
            return None
        for _t in range(8):
            y = int(nb[int(rng.integers(0, d))])
            if y not in excl:
                return y
        rest = [int(y) for y in nb if int(y) not in excl]
        return rest[int(rng.integers(0, len(rest)))] if rest else None

    def adjacent(u, v):
        nb = g.neighbors(u)
        j = int(np.searchsorted(nb, v))
        return j < nb.shape[0] and int(nb[j]) == v

    for _ in range(max_tries):
        start = int(rng.integers(0, nv))
        if deg[start] == 0:
            continue
        if shape == "cycle":
            path = [start]
            seen = {start}
            while len(path) < k:
                y = rand_nb(path[-1], seen)
                if y is None:
                    break
                path.append(y)
                seen.add(y)
            if len(path) < k or not adjacent(path[-1], path[0]):
                continue
            verts = path
            edges_local = [(i, i + 1) for i in range(k - 1)] + [(k - 1, 0)]
        else:
            verts = [start]
            vset = {start}
            frontier = [start]
            while len(verts) < k and frontier:
                x = frontier[int(rng.integers(0, len(frontier)))]
                y = rand_nb(x, vset)
                if y is None:
                    frontier.remove(x)
                    continue
                verts.append(y)
                vset.add(y)
                frontier.append(y)
            if len(verts) < k:
                continue
            varr = np.asarray(verts, dtype=np.int64)
            induced = []
            for i, v in enumerate(verts):
                nb = g.neighbors(v)
                j = np.minimum(np.searchsorted(nb, varr), max(nb.shape[0] - 1, 0))
                hit = (nb.shape[0] > 0) & (nb[j] == varr) if nb.shape[0] else np.zeros(k, dtype=bool)
                for jj in np.nonzero(hit)[0]:
                    if i < int(jj):
                        induced.append((i, int(jj)))
            # random spanning tree of the induced subgraph (randomised Kruskal)
            order = rng.permutation(len(induced))
            parent = list(range(k))

            def find(x):
                while parent[x] != x:
                    parent[x] = parent[parent[x]]
                    x = parent[x]
                return x

            tree, rest = [], []
            for oi in order:
                a, b = induced[int(oi)]
                ra, rb = find(a), find(b)
                if ra != rb:
                    parent[ra] = rb
                    tree.append((a, b))
                else:
                    rest.append((a, b))
            if len(tree) != k - 1:
                continue
            edges_local = list(tree)
            if shape == "chord":
                if not rest:
                    continue
                edges_local.append(rest[int(rng.integers(0, len(rest)))])
        labels = [int(g.vlabel[v]) for v in verts]
        elabs = [_edge_label(g, verts[a], verts[b]) for a, b in edges_local]
        rare = min(range(k), key=lambda i: (vcount[labels[i]], i))
        order = _bfs_number(k, edges_local, rare)
        newid = {old: new for new, old in enumerate(order)}
        return Pattern(vlabel=[labels[o] for o in order],
                       edges=[(newid[a], newid[b]) for a, b in edges_local],
                       elabel=list(elabs))
    return None


def sample_patterns(g: Graph, count: int, seed: int, kmin: int = 3, kmax: int = 7,
                    shapes=("tree", "cycle", "chord")) -> List[Pattern]:
    rng = np.random.default_rng(seed)
    out: List[Pattern] = []
    while len(out) < count:
        k = int(rng.integers(kmin, kmax + 1))
        shape = shapes[int(rng.integers(0, len(shapes)))]
        p = sample_pattern(g, rng, k, shape)
        if p is not None:
            out.append(p)
    return out


def random_connected_pattern(rng: np.random.Generator, n: int, n_vlabels: int, n_elabels: int,
                             extra_edge_p: float = 0.3, prefix_connected: bool = True) -> Pattern:
    """A random connected labeled pattern on n vertices (for tiny cross-checks).

    With prefix_connected=False the vertex numbering is shuffled, so a vertex
    may have no earlier neighbour.
    """
    edges = set()
    for i in range(1, n):
        j = int(rng.integers(0, i))
        edges.add((j, i))
    for i in range(n):
        for j in range(i + 1, n):
            if (i, j) not in edges and rng.random() < extra_edge_p:
                edges.add((i, j))
    edges = sorted(edges)
    if not prefix_connected:
        perm = rng.permutation(n)
        edges = sorted((min(int(perm[a]), int(perm[b])), max(int(perm[a]), int(perm[b]))) for a, b in edges)
    vl = [int(x) for x in rng.integers(0, n_vlabels, size=n)]
    el = [int(x) for x in rng.integers(0, n_elabels, size=len(edges))] if n_elabels > 1 else [0] * len(edges)
    return Pattern(vlabel=vl, edges=list(edges), elabel=el)
