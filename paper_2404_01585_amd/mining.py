"""Level-wise mining driver (host side) around the support query.

This is the loop of Algorithm 1 (mining: candidates -> tau -> matcher ->
next candidates) with a plain one-edge extension generator standing in for
the paper's vertex-merge generator (Algorithms 2-4):

* level 1: every distinct labeled edge of the data graph (``edges(G)`` in
  Algorithm 1);
* level k+1: every frequent k-edge pattern extended by one edge -- to a new
  vertex (forward) or between two existing vertices (backward) -- with the
  label combination of the added edge itself frequent at level 1;
* a candidate is kept only if every connected sub-pattern with one edge
  fewer is frequent (the anti-monotone pruning of Section 2.2.1) and if n
  disjoint images could fit in the graph (the size bound of Section 3.1.2);
* duplicates are removed by a canonical form computed by brute force over
  vertex orders that respect a vertex invariant (patterns here have at most
  a handful of vertices).

Patterns are submitted numbered in BFS order from canonical vertex 0, so
every prefix of the numbering is connected.

The support function is a callback, so the same candidate lists drive the
device path and the oracle.
"""

from __future__ import annotations

import functools
import itertools
from collections import deque
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

from .synth import Graph, Pattern

Key = Tuple[Tuple[int, ...], Tuple[Tuple[int, int, int], ...]]


def _adj(n: int, edges: Sequence[Tuple[int, int]], elabel: Sequence[int]):
    adj = [dict() for _ in range(n)]
    for (a, b), l in zip(edges, elabel):
        adj[a][b] = l
        adj[b][a] = l
    return adj


def canonical_key(p: Pattern) -> Tuple[Key, List[int]]:
    """Smallest (labels, sorted edge list) encoding over invariant-respecting
    vertex orders, and the order (old ids in canonical position order)."""
    key, perm = _canonical_key(tuple(p.vlabel), tuple(tuple(e) for e in p.edges), tuple(p.elabel))
    return key, list(perm)


@functools.lru_cache(maxsize=1 << 20)
def _canonical_key(vlabel, edges, elabel):
    p = Pattern(vlabel=list(vlabel), edges=[tuple(e) for e in edges], elabel=list(elabel))
    n = p.n
    adj = _adj(n, p.edges, p.elabel)
    inv = [(p.vlabel[v], len(adj[v]), tuple(sorted((p.vlabel[u], l) for u, l in adj[v].items()))) for v in range(n)]
    order = sorted(range(n), key=lambda v: inv[v])
    cells: List[List[int]] = []
    for v in order:
        if cells and inv[cells[-1][0]] == inv[v]:
            cells[-1].append(v)
        else:
            cells.append([v])
    best: Optional[Key] = None
    best_perm: List[int] = []
    for choice in itertools.product(*[itertools.permutations(c) for c in cells]):
        perm = [v for c in choice for v in c]  # position -> old vertex
        pos = {v: i for i, v in enumerate(perm)}
        labels = tuple(p.vlabel[v] for v in perm)
        es = tuple(sorted((min(pos[a], pos[b]), max(pos[a], pos[b]), l) for (a, b), l in zip(p.edges, p.elabel)))
        key = (labels, es)
        if best is None or key < best:
            best, best_perm = key, perm
    return best, tuple(best_perm)


def from_key(key: Key) -> Pattern:
    """Pattern numbered in BFS order from canonical vertex 0 (connected prefixes)."""
    labels, es = key
    n = len(labels)
    adj = [[] for _ in range(n)]
    for a, b, _ in es:
        adj[a].append(b)
        adj[b].append(a)
    seen = [False] * n
    order = []
    dq = deque([0])
    seen[0] = True
    while dq:
        x = dq.popleft()
        order.append(x)
        for y in sorted(adj[x]):
            if not seen[y]:
                seen[y] = True
                dq.append(y)
    new = {old: i for i, old in enumerate(order)}
    return Pattern(vlabel=[labels[o] for o in order], edges=[(new[a], new[b]) for a, b, _ in es],
                   elabel=[l for _, _, l in es])


def edge_types(g: Graph) -> List[Tuple[int, int, int]]:
    """Distinct (label_a <= label_b, edge label) of the data graph's edges."""
    el = g.edge_list()
    la = g.vlabel[el[:, 0]].astype(np.int64)
    lb = g.vlabel[el[:, 1]].astype(np.int64)
    lo, hi = np.minimum(la, lb), np.maximum(la, lb)
    trip = np.unique(np.stack([lo, hi, el[:, 2]], axis=1), axis=0)
    return [tuple(int(x) for x in t) for t in trip]


def _is_connected(n: int, edges: Sequence[Tuple[int, int]]) -> bool:
    if n == 1:
        return True
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = {0}
    st = [0]
    while st:
        x = st.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                st.append(y)
    return len(seen) == n


def sub_patterns(p: Pattern) -> Iterable[Pattern]:
    """Connected patterns with one edge fewer (an isolated vertex is removed)."""
    for k in range(p.m):
        edges = [e for i, e in enumerate(p.edges) if i != k]
        labs = [l for i, l in enumerate(p.elabel) if i != k]
        deg = [0] * p.n
        for a, b in edges:
            deg[a] += 1
            deg[b] += 1
        keep = [v for v in range(p.n) if deg[v] > 0 or p.n == 1]
        if len(keep) < p.n - 1 or not edges:
            continue
        idx = {v: i for i, v in enumerate(keep)}
        q = Pattern(vlabel=[p.vlabel[v] for v in keep], edges=[(idx[a], idx[b]) for a, b in edges], elabel=labs)
        if _is_connected(q.n, q.edges):
            yield q


def extensions(p: Pattern, freq_types: set, max_vertices: int) -> Iterable[Pattern]:
    adj = _adj(p.n, p.edges, p.elabel)
    labels_by = {}
    for a, b, e in freq_types:
        labels_by.setdefault(a, set()).add((b, e))
        labels_by.setdefault(b, set()).add((a, e))
    if p.n < max_vertices:
        for u in range(p.n):
            for lab, e in sorted(labels_by.get(p.vlabel[u], ())):
                yield Pattern(vlabel=p.vlabel + [lab], edges=p.edges + [(u, p.n)], elabel=p.elabel + [e])
    for u in range(p.n):
        for v in range(u + 1, p.n):
            if v in adj[u]:
                continue
            a, b = sorted((p.vlabel[u], p.vlabel[v]))
            for e in sorted({e for (x, y, e) in freq_types if x == a and y == b}):
                yield Pattern(vlabel=list(p.vlabel), edges=p.edges + [(u, v)], elabel=p.elabel + [e])


SupportFn = Callable[[List[Pattern], int, float], List[Dict]]


def mine(g: Graph, sigma: int, lam: float, max_edges: int, evaluate: SupportFn,
         max_vertices: int = 16, max_candidates: Optional[int] = None, tau_fn=None,
         types: Optional[List[Tuple[int, int, int]]] = None, evaluate_last: bool = True) -> Dict:
    """Runs the level-wise loop.  ``evaluate(patterns, sigma, lam)`` returns one
    result dict per pattern with at least 'frequent'.  Returns the candidate
    lists and results of every level.  ``types``: the graph's edge types
    (``edge_types(g)``), when the caller already has them.  With
    ``evaluate_last`` false the candidates of level ``max_edges`` are generated
    but not evaluated (their results list is empty)."""
    nv = g.num_vertices
    if types is None:
        types = edge_types(g)
    level_cands: List[List[Pattern]] = []
    level_res: List[List[Dict]] = []
    cands = [from_key(canonical_key(Pattern([a, b], [(0, 1)], [e]))[0]) for a, b, e in types]
    freq_keys: set = set()
    freq_types: set = set()
    for level in range(1, max_edges + 1):
        if not cands:
            break
        if max_candidates is not None:
            cands = cands[:max_candidates]
        if level == max_edges and not evaluate_last:
            level_cands.append(cands)
            level_res.append([])
            break
        res = evaluate(cands, sigma, lam)
        level_cands.append(cands)
        level_res.append(res)
        frequent = [p for p, r in zip(cands, res) if r["frequent"]]
        for p in frequent:
            freq_keys.add(canonical_key(p)[0])
        if level == 1:
            for p in frequent:
                a, b = sorted(p.vlabel)
                freq_types.add((a, b, p.elabel[0]))
        if level == max_edges:
            break
        seen = set()
        nxt = []
        for p in frequent:
            for q in extensions(p, freq_types, max_vertices):
                key, _ = canonical_key(q)
                if key in seen:
                    continue
                seen.add(key)
                qq = from_key(key)
                if tau_fn is not None and qq.n * max(tau_fn(sigma, lam, qq.n), 1) > nv:
                    continue  # n * tau <= |V| bound
                if all(canonical_key(s)[0] in freq_keys for s in sub_patterns(qq)):
                    nxt.append(qq)
        nxt.sort(key=lambda p: canonical_key(p)[0])
        cands = nxt
    return dict(levels=level_cands, results=level_res)
