"""Candidate generation by merging core graphs (Section 3.2.1, Algorithms 2-4).

k-vertex candidates come from pairs of frequent (k-1)-vertex patterns:

* a core graph of a pattern P is P with one vertex u disconnected (Section
  2.3: the marked vertex); its core is P - u, possibly disconnected;
* core graphs are grouped by the isomorphism class of their core (core
  groups), each expressed in its core's canonical vertex order, so that the
  marked vertex's attachment -- the (core vertex, edge label) pairs it was
  joined to -- is comparable across the group;
* merging two core graphs of a group puts both marked vertices back on one
  copy of the core; the core's automorphisms give the different relative
  placements (Algorithm 3: when an attachment is invariant under every
  automorphism there is only one placement);
* the two marked vertices are never joined, so cliques need a third pattern
  for the missing edge (Algorithm 4); a clique candidate is kept only if all
  of its (k-1)-vertex sub-cliques are frequent;
* duplicates are removed by canonical form (Algorithm 2, RemoveDuplicates).

Every connected non-clique k-vertex pattern has two non-adjacent vertices
whose removals leave it connected (the non-articulation lemma of Section
3.2.1), so every such pattern whose two (k-1)-vertex sub-patterns are
frequent is produced.  Canonical forms are computed by brute force over
vertex orders (patterns have a handful of vertices), standing in for Bliss.
"""

from __future__ import annotations

import itertools
from collections import defaultdict
from typing import Dict, Iterable, List, Optional, Sequence, Set, Tuple

from .mining import Key, canonical_key, edge_types, from_key
from .synth import Graph, Pattern

Attach = Tuple[Tuple[int, int], ...]  # sorted (core position, edge label)


def _remove_vertex(p: Pattern, u: int) -> Tuple[Pattern, Dict[int, int], List[Tuple[int, int]]]:
    """P - u (vertices renumbered in order), the old -> new map, and u's
    attachment as (new id, edge label)."""
    keep = [v for v in range(p.n) if v != u]
    idx = {v: i for i, v in enumerate(keep)}
    edges, labs, att = [], [], []
    for (a, b), l in zip(p.edges, p.elabel):
        if a == u:
            att.append((idx[b], l))
        elif b == u:
            att.append((idx[a], l))
        else:
            edges.append((idx[a], idx[b]))
            labs.append(l)
    return Pattern(vlabel=[p.vlabel[v] for v in keep], edges=edges, elabel=labs), idx, att


def _key_pattern(key: Key) -> Pattern:
    """The pattern of a canonical key, numbered in canonical position order
    (unlike from_key, which renumbers in BFS order)."""
    labels, es = key
    return Pattern(vlabel=list(labels), edges=[(a, b) for a, b, _ in es], elabel=[l for _, _, l in es])


def automorphisms(key: Key) -> List[Tuple[int, ...]]:
    """Automorphisms of the canonical pattern `key` as position permutations
    (alpha[i] = image of position i).  Brute force over label-preserving
    permutations, pruned by degree."""
    labels, es = key
    n = len(labels)
    eset = {(a, b): l for a, b, l in es}
    deg = [0] * n
    for a, b, _ in es:
        deg[a] += 1
        deg[b] += 1
    cls = defaultdict(list)
    for v in range(n):
        cls[(labels[v], deg[v])].append(v)
    groups = list(cls.values())
    out = []
    for choice in itertools.product(*[itertools.permutations(gr) for gr in groups]):
        alpha = [0] * n
        for gr, img in zip(groups, choice):
            for a, b in zip(gr, img):
                alpha[a] = b
        ok = True
        for (a, b), l in eset.items():
            x, y = alpha[a], alpha[b]
            if eset.get((min(x, y), max(x, y))) != l:
                ok = False
                break
        if ok:
            out.append(tuple(alpha))
    return out


class CoreGraph:
    __slots__ = ("parent", "label", "attach", "parent_clique")

    def __init__(self, parent: Key, label: int, attach: Attach, parent_clique: bool):
        self.parent = parent
        self.label = label
        self.attach = attach
        self.parent_clique = parent_clique


def _is_clique(p: Pattern) -> bool:
    return p.m == p.n * (p.n - 1) // 2


def core_groups(patterns: Sequence[Pattern]) -> Dict[Key, List[CoreGraph]]:
    """Core groups (Section 2.3) of a set of same-size patterns: core key ->
    core graphs, attachments in the core's canonical positions."""
    groups: Dict[Key, List[CoreGraph]] = defaultdict(list)
    for p in patterns:
        pkey = canonical_key(p)[0]
        clique = _is_clique(p)
        for u in range(p.n):
            core, _, att = _remove_vertex(p, u)
            ckey, perm = canonical_key(core)
            pos = {old: i for i, old in enumerate(perm)}
            attach = tuple(sorted((pos[v], l) for v, l in att))
            groups[ckey].append(CoreGraph(pkey, p.vlabel[u], attach, clique))
    return groups


def _merge(core: Key, a: CoreGraph, b_attach: Attach, b_label: int) -> Pattern:
    """The core plus both marked vertices: a's at position m, b's at m + 1."""
    labels, es = core
    m = len(labels)
    edges = [(x, y) for x, y, _ in es]
    elab = [l for _, _, l in es]
    for v, l in a.attach:
        edges.append((v, m))
        elab.append(l)
    for v, l in b_attach:
        edges.append((v, m + 1))
        elab.append(l)
    return Pattern(vlabel=list(labels) + [a.label, b_label], edges=edges, elabel=elab)


def generate_new_patterns(frequent: Sequence[Pattern], edge_labels: Optional[Dict[Tuple[int, int], Set[int]]] = None
                          ) -> List[Pattern]:
    """k-vertex candidates from the frequent (k-1)-vertex patterns (Algorithm 2).

    edge_labels: for the clique step, the edge labels a (label, label) pair
    may carry (the frequent labeled edges); None takes every edge label that
    occurs in `frequent`."""
    if not frequent:
        return []
    freq_keys = {canonical_key(p)[0] for p in frequent}
    if edge_labels is None:
        all_l = {l for p in frequent for l in p.elabel}
        edge_labels = defaultdict(lambda: all_l)
    out: Dict[Key, Pattern] = {}

    def add(q: Pattern):
        k = canonical_key(q)[0]
        if k not in out:
            out[k] = from_key(k)

    for core, members in core_groups(frequent).items():
        auts = automorphisms(core)
        for i in range(len(members)):
            for j in range(i, len(members)):
                a, b = members[i], members[j]
                # Algorithm 3: every distinct placement of b's attachment
                placements = {tuple(sorted((alpha[v], l) for v, l in b.attach)) for alpha in auts}
                for batt in sorted(placements):
                    merged = _merge(core, a, batt, b.label)
                    add(merged)
                    # Algorithm 4: two cliques whose marked vertices see the whole
                    # core leave only the edge between the marked vertices missing
                    m = len(core[0])
                    if a.parent_clique and b.parent_clique and len(a.attach) == m and len(batt) == m:
                        lo, hi = sorted((a.label, b.label))
                        for e in sorted(edge_labels[(lo, hi)]):
                            clique = Pattern(vlabel=merged.vlabel, edges=merged.edges + [(m, m + 1)],
                                             elabel=merged.elabel + [e])
                            # every (k-1)-vertex sub-clique must be frequent
                            if all(canonical_key(_remove_vertex(clique, w)[0])[0] in freq_keys
                                   for w in range(clique.n)):
                                add(clique)
    return [out[k] for k in sorted(out)]


def edge_patterns(g: Graph) -> List[Pattern]:
    """The 2-vertex candidates: every distinct labeled edge of the data graph
    (edges(G) of Algorithm 1)."""
    return [from_key(canonical_key(Pattern([a, b], [(0, 1)], [e]))[0]) for a, b, e in edge_types(g)]


def mine_by_vertices(g: Graph, sigma: int, lam: float, max_vertices: int, evaluate, tau_fn) -> Dict:
    """Algorithm 1 with the merge generator: levels by vertex count, from the
    labeled edges, while candidates remain and n * tau fits in the graph
    (Section 3.1.2).  ``evaluate(patterns, sigma, lam)`` returns one result
    per pattern with at least 'frequent'."""
    nv = g.num_vertices
    levels, results = [], []
    cands = edge_patterns(g)
    freq_edges: Dict[Tuple[int, int], Set[int]] = defaultdict(set)
    n = 2
    while cands and n <= max_vertices:
        if n * max(tau_fn(sigma, lam, n), 1) > nv:
            break
        res = evaluate(cands, sigma, lam)
        levels.append(cands)
        results.append(res)
        frequent = [p for p, r in zip(cands, res) if r["frequent"]]
        if n == 2:
            for p in frequent:
                lo, hi = sorted(p.vlabel)
                freq_edges[(lo, hi)].add(p.elabel[0])
        n += 1
        cands = generate_new_patterns(frequent, freq_edges) if n <= max_vertices else []
    return {"levels": levels, "results": results}
