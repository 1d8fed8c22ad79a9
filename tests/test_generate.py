"""The merge-based candidate generator (Section 3.2.1, Algorithms 2-4).

Pinned against the paper's worked merges (Examples 1 and 2) and against
its definition, by brute force over every small labeled pattern: the
candidates from a set F of frequent (k-1)-vertex patterns are exactly the
connected k-vertex patterns with two non-adjacent vertices u, v such that
P - u and P - v are in F, plus the k-cliques all of whose (k-1)-vertex
sub-cliques are in F."""

import itertools

import numpy as np
import pytest

from helpers import load_fixture
from oracle import oracle as O
from paper_2404_01585_amd import generate as G
from paper_2404_01585_amd import mining
from paper_2404_01585_amd.synth import Pattern, tiny_random_graph


def key(p):
    return mining.canonical_key(p)[0]


def keys(ps):
    return {key(p) for p in ps}


def test_paper_examples():
    run = load_fixture("running_example.txt")
    ex = load_fixture("merge_examples.txt")
    got = keys(G.generate_new_patterns([run["P1"], run["P2"]]))
    for name in ("E1a", "E1b", "E1c"):
        assert key(ex[name]) in got, name
    got = keys(G.generate_new_patterns([ex["P"]]))
    assert key(ex["E2a"]) in got and key(ex["E2b"]) in got
    assert key(ex["E2a"]) != key(ex["E2b"])


def test_automorphisms_of_known_shapes():
    tri = key(Pattern([0, 0, 0], [(0, 1), (1, 2), (0, 2)], [0, 0, 0]))
    assert len(G.automorphisms(tri)) == 6
    path = key(Pattern([0, 0, 0], [(0, 1), (1, 2)], [0, 0]))
    assert len(G.automorphisms(path)) == 2
    c4 = key(Pattern([0, 0, 0, 0], [(0, 1), (1, 2), (2, 3), (3, 0)], [0] * 4))
    assert len(G.automorphisms(c4)) == 8  # the dihedral group of the square
    lab = key(Pattern([0, 1, 0], [(0, 1), (1, 2)], [0, 1]))
    assert len(G.automorphisms(lab)) == 1  # edge labels break the mirror


def _all_patterns(n, nvl, nel):
    """Every connected labeled pattern on n vertices, up to isomorphism."""
    pairs = list(itertools.combinations(range(n), 2))
    out = {}
    for vl in itertools.product(range(nvl), repeat=n):
        for choice in itertools.product(range(nel + 1), repeat=len(pairs)):
            es = [(a, b) for (a, b), c in zip(pairs, choice) if c]
            if not es or not mining._is_connected(n, es):
                continue
            p = Pattern(list(vl), es, [c - 1 for c in choice if c])
            out.setdefault(key(p), p)
    return out


def _definition(cands_k, freq_keys):
    want = set()
    for k, p in cands_k.items():
        adj = {(min(a, b), max(a, b)) for a, b in p.edges}
        sub = [key(G._remove_vertex(p, w)[0]) for w in range(p.n)]
        if len(adj) == p.n * (p.n - 1) // 2:
            if all(s in freq_keys for s in sub):
                want.add(k)
            continue
        for u, v in itertools.combinations(range(p.n), 2):
            if (u, v) not in adj and sub[u] in freq_keys and sub[v] in freq_keys:
                want.add(k)
                break
    return want


@pytest.mark.parametrize("n,nvl,nel", [(3, 2, 1), (3, 2, 2), (4, 2, 1), (4, 1, 2), (5, 1, 1)])
def test_matches_definition(n, nvl, nel):
    small = _all_patterns(n - 1, nvl, nel)
    big = _all_patterns(n, nvl, nel)
    rng = np.random.default_rng(100 * n + 10 * nvl + nel)
    for trial in range(6):
        frac = [1.0, 0.8, 0.5, 0.3][trial % 4]
        fk = {k for k in small if rng.random() < frac}
        got = keys(G.generate_new_patterns([small[k] for k in sorted(fk)]))
        assert got == _definition(big, fk), (n, nvl, nel, trial)


def test_mining_by_vertices_on_tiny_graphs():
    """Algorithm 1 with the merge generator and the oracle's verdicts: every
    candidate of level n+1 is justified by the frequent patterns of level n
    (two frequent vertex-deleted sub-patterns at non-adjacent vertices, or
    all of them for a clique), no two candidates are isomorphic, and the
    levels stop once n * tau exceeds the graph (Section 3.1.2)."""
    rng = np.random.default_rng(8)
    for _ in range(6):
        g = tiny_random_graph(rng, 24, 0.25, 2, 2)

        def ev(ps, s, l):
            return [O.query(g, p, s, l, mode=O.VERDICT) for p in ps]

        r = G.mine_by_vertices(g, 2, 1.0, 5, ev, O.tau)
        assert [len(set(keys(c))) for c in r["levels"]] == [len(c) for c in r["levels"]]
        for lv in range(1, len(r["levels"])):
            prev = {key(p) for p, x in zip(r["levels"][lv - 1], r["results"][lv - 1]) if x["frequent"]}
            cur = {key(p): p for p in r["levels"][lv]}
            assert set(cur) <= _definition(cur, prev)
        for c in r["levels"]:
            n = c[0].n
            assert n * max(O.tau(2, 1.0, n), 1) <= g.num_vertices
