"""Shared test helpers: golden-fixture parsing and small graph utilities."""

import os
from typing import Dict, List, Tuple

import numpy as np

from paper_2404_01585_amd.synth import Graph, Pattern, csr_from_edges

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _pairs(vals: List[int]) -> List[Tuple[int, int]]:
    return [(vals[i], vals[i + 1]) for i in range(0, len(vals), 2)]


def load_fixture(name: str) -> Dict[str, object]:
    """Parses a golden .txt file into {name: Graph | Pattern}."""
    out: Dict[str, object] = {}
    cur = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] in ("graph", "pattern"):
                cur = {"kind": tok[0], "name": tok[1]}
            elif tok[0] == "end":
                if cur["kind"] == "graph":
                    nv = cur["vertices"]
                    e = _pairs(cur["edges"])
                    el = cur.get("elabels", [0] * len(e))
                    g = csr_from_edges(nv, [a for a, _ in e], [b for _, b in e], el, cur["vlabels"],
                                       offset_dtype=np.int64, name=cur["name"])
                    out[cur["name"]] = g
                else:
                    e = _pairs(cur["edges"])
                    out[cur["name"]] = Pattern(vlabel=cur["vlabels"], edges=e,
                                               elabel=cur.get("elabels", [0] * len(e)))
                cur = None
            else:
                vals = [int(x) for x in tok[1:]]
                cur[tok[0]] = vals[0] if tok[0] == "vertices" else vals
    return out


def load_expected(name: str) -> Dict[Tuple[str, str], List[str]]:
    out = {}
    taus = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "tau":
                taus.append((int(tok[1]), float(tok[2]), int(tok[3])))
            else:
                out[(tok[0], tok[1])] = tok[2:]
    out[("tau", "cases")] = taus
    return out


def adjacency_matrix(g: Graph) -> np.ndarray:
    nv = g.num_vertices
    a = np.zeros((nv, nv), dtype=np.int64)
    src = np.repeat(np.arange(nv), g.degree())
    a[src, g.col] = 1
    return a


def relabel_all(g: Graph, label: int = 0) -> Graph:
    return Graph(row_ptr=g.row_ptr, col=g.col, vlabel=np.full_like(g.vlabel, label),
                 elabel=np.zeros_like(g.elabel), name=g.name + "_unlabeled")


def automorphisms(p: Pattern) -> int:
    """Number of label- and edge-preserving permutations of the pattern (brute force)."""
    import itertools
    n = p.n
    E = {}
    for (a, b), l in zip(p.edges, p.elabel):
        E[(a, b)] = l
        E[(b, a)] = l
    cnt = 0
    for perm in itertools.permutations(range(n)):
        if any(p.vlabel[perm[i]] != p.vlabel[i] for i in range(n)):
            continue
        if all(E.get((perm[a], perm[b])) == l for (a, b), l in zip(p.edges, p.elabel)):
            cnt += 1
    return cnt
