"""Symmetry breaking of the support phase, tested on the CPU: the masks the
library derives (paper_2404_01585_amd/csrc/fx_sym.h, built with the host
compiler) against the same construction done by brute force over all vertex
permutations, and the property that makes them exact: in every automorphism
orbit of embeddings exactly one member meets the constraints, its
lexicographically smallest (checked against the oracle's embedding lists on
tiny graphs)."""

import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2404_01585_amd.synth import Pattern, random_connected_pattern, tiny_random_graph

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _automorphisms(p):
    e = {}
    for (a, b), l in zip(p.edges, p.elabel):
        e[(a, b)] = l
        e[(b, a)] = l
    out = []
    for perm in itertools.permutations(range(p.n)):
        if any(p.vlabel[i] != p.vlabel[perm[i]] for i in range(p.n)):
            continue
        if all(e.get((perm[a], perm[b])) == l for (a, b), l in e.items()):
            out.append(perm)
    return out


def _brute_masks(p):
    group = _automorphisms(p)
    lt = [0] * p.n
    for v in range(p.n):
        for w in sorted({a[v] for a in group} - {v}):
            assert w > v
            lt[w] |= 1 << v
        group = [a for a in group if a[v] == v]
    return lt


@pytest.fixture(scope="module")
def sym_exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("sym") / "sym_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_2404_01585_amd", "csrc"),
                           os.path.join(HERE, "host_sym_test.cpp"), "-o", exe])
    return exe


def _run(exe, pats, budget=0):
    lines = [str(len(pats))]
    for p in pats:
        el = [[-1] * p.n for _ in range(p.n)]
        for (a, b), l in zip(p.edges, p.elabel):
            el[a][b] = el[b][a] = l
        lines.append(" ".join(map(str, [budget, p.n] + list(p.vlabel) + [x for row in el for x in row])))
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    return [list(map(int, ln.split())) for ln in out.stdout.strip().splitlines()]


def test_masks_match_brute_force(sym_exe):
    rng = np.random.default_rng(11)
    pats = []
    for _ in range(300):
        n = int(rng.integers(1, 8))
        pats.append(random_connected_pattern(rng, n, int(rng.integers(1, 4)), int(rng.integers(1, 3)),
                                             extra_edge_p=float(rng.uniform(0.0, 0.7)),
                                             prefix_connected=bool(rng.random() < 0.7)))
    # shapes with large groups: cycles, a complete graph, a star (in several numberings)
    pats.append(Pattern([0] * 6, [(i, (i + 1) % 6) for i in range(6)], [0] * 6))
    pats.append(Pattern([0] * 5, [(i, j) for i in range(5) for j in range(i + 1, 5)], [0] * 10))
    pats.append(Pattern([0] * 6, [(2, j) for j in range(6) if j != 2], [0] * 5))
    got = _run(sym_exe, pats)
    for p, g in zip(pats, got):
        assert g == _brute_masks(p), (p, g)
    assert sum(any(m) for m in got) > 50  # many of them are symmetric


def test_star16_chain(sym_exe):
    # a 16-vertex star with equal labels: the leaves must come in increasing order
    star = Pattern([0] * 16, [(0, j) for j in range(1, 16)], [0] * 15)
    (got,) = _run(sym_exe, [star])
    assert got[0] == 0 and got[1] == 0
    for w in range(2, 16):
        assert got[w] == sum(1 << v for v in range(1, w))


def test_constraints_keep_the_smallest_of_each_orbit(sym_exe):
    rng = np.random.default_rng(5)
    cases = []
    while len(cases) < 150:
        n = int(rng.integers(2, 6))
        nvl = int(rng.integers(1, 3))
        p = random_connected_pattern(rng, n, nvl, 1, extra_edge_p=0.4, prefix_connected=bool(rng.random() < 0.7))
        g = tiny_random_graph(rng, int(rng.integers(5, 14)), 0.4, nvl, 1)
        cases.append((p, g))
    masks = _run(sym_exe, [p for p, _ in cases])
    nonempty = 0
    for (p, g), lt in zip(cases, masks):
        cnt, rows = O.enumerate_embeddings(g, p, cap=1 << 20)
        group = _automorphisms(p)
        for r in map(tuple, rows):
            orbit = {tuple(r[a[i]] for i in range(p.n)) for a in group}
            meets = all(not ((lt[w] >> v) & 1) or r[v] < r[w] for w in range(p.n) for v in range(p.n))
            assert meets == (r == min(orbit)), (p, r, lt)
        nonempty += cnt > 0 and any(lt)
    assert nonempty > 20


def test_cut_short_search_keeps_a_subset(sym_exe):
    # with a tiny search budget the masks are a subset of the full ones (every
    # kept constraint is one the smallest member meets), never something else
    rng = np.random.default_rng(12)
    pats = [random_connected_pattern(rng, int(rng.integers(3, 8)), 1, 1, extra_edge_p=0.3) for _ in range(120)]
    full = _run(sym_exe, pats)
    for budget in (1, 5, 20, 60):
        part = _run(sym_exe, pats, budget)
        for f, g in zip(full, part):
            assert all((x & y) == x for x, y in zip(g, f)), (budget, f, g)
        assert sum(map(sum, part)) <= sum(map(sum, full))
    assert _run(sym_exe, pats, 1) != full  # the budget does cut


def test_rigid_sixteen_vertex_pattern_returns(sym_exe):
    # a 16-vertex pattern with one label and no symmetry: the search ends (by
    # exhausting it or the budget) and keeps no constraint
    edges = [(i, i + 1) for i in range(15)] + [(0, 2), (1, 4), (3, 7), (5, 11)]
    rigid = Pattern([0] * 16, edges, [0] * len(edges))
    (got,) = _run(sym_exe, [rigid])
    assert got == [0] * 16
