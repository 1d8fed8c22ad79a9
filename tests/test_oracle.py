"""Pins of the CPU oracle against values the paper prints, closed forms,
invariants and brute force (no GPU)."""

import math

import numpy as np
import pytest

from helpers import adjacency_matrix, automorphisms, load_expected, load_fixture, relabel_all
from oracle import oracle as O
from paper_2404_01585_amd.synth import Pattern, random_connected_pattern, tiny_random_graph


@pytest.fixture(scope="module")
def running():
    return load_fixture("running_example.txt"), load_expected("running_example.expected")


@pytest.fixture(scope="module")
def tight():
    return load_fixture("tight_bound.txt"), load_expected("tight_bound.expected")


# ---------------------------------------------------------------------------
# tau (Section 3.1.1)
# ---------------------------------------------------------------------------

def test_tau_printed_cases(running):
    _, exp = running
    for sigma, lam, t in exp[("tau", "cases")]:
        assert O.tau(sigma, lam, 3) == t


@pytest.mark.parametrize("sigma", [1, 2, 7, 20, 57, 200, 1600, 2000, 123457])
@pytest.mark.parametrize("n", [2, 3, 4, 5, 8, 16])
def test_tau_endpoints(sigma, n):
    # the paper: lambda = 1 gives tau = sigma, lambda = 0 gives sigma / n
    assert O.tau(sigma, 1.0, n) == sigma
    assert O.tau(sigma, 0.0, n) == sigma // n


def test_tau_exact_where_doubles_round_wrong():
    # 375 * (4 * 0.57 + 1) / 5 = 375 * 3.28 / 5 = 246 exactly; the double
    # expression sigma*(1-1/n)*lambda + sigma/n evaluates to 245.999...
    assert 375 * (1 - 1 / 5) * 0.57 + 375 / 5 < 246
    assert O.tau(375, 0.57, 5) == 246
    # 3550 * (6 * 0.37 + 1) / 7 = 3550 * 3.22 / 7 = 1633 exactly
    assert O.tau(3550, 0.37, 7) == 1633


def test_tau_monotone_in_lambda():
    for n in (2, 3, 5, 8):
        prev = -1
        for k in range(0, 101):
            t = O.tau(997, k / 100, n)
            assert t >= prev
            prev = t


# ---------------------------------------------------------------------------
# Running example (Section 2.1.3, Section 2.2, Section 2.4, Section 3.1.1)
# ---------------------------------------------------------------------------

def test_running_example_mappings(running):
    fx, exp = running
    D, P1 = fx["D"], fx["P1"]
    printed = [int(x) for x in exp[("P1", "mappings")]]
    printed = sorted(tuple(printed[i:i + 3]) for i in range(0, len(printed), 3))
    cnt, rows = O.enumerate_embeddings(D, P1)
    assert cnt == 6
    assert [tuple(r) for r in rows.tolist()] == printed
    assert O.brute_embeddings(D, P1) == printed


def test_running_example_metrics(running):
    fx, exp = running
    D, P1 = fx["D"], fx["P1"]
    embs = O.brute_embeddings(D, P1)
    assert O.brute_mis(embs) == int(exp[("P1", "mis")][0])
    assert O.mni(D, P1) == int(exp[("P1", "mni")][0])
    assert O.brute_mni(embs, 3) == int(exp[("P1", "mni")][0])
    lo, hi = (int(x) for x in exp[("P1", "mis_maximal_range")])
    k, sel = O.support_stream(D, P1)
    assert lo <= k <= hi
    # lexicographic greedy picks Mapping IV: (d1,d5,d2) and (d3,d7,d4)
    assert k == 2
    assert [tuple(r) for r in sel.tolist()] == [(0, 4, 1), (2, 6, 3)]
    assert O.is_maximal_independent([tuple(r) for r in sel.tolist()], embs)
    # automorphisms: 2 with labels, 6 when unlabeled; |Aut| divides |M|
    assert automorphisms(P1) == int(exp[("P1", "automorphisms")][0])
    P1u = Pattern(vlabel=[0, 0, 0], edges=P1.edges, elabel=P1.elabel)
    assert automorphisms(P1u) == int(exp[("P1_unlabeled", "automorphisms")][0])
    assert len(embs) % automorphisms(P1) == 0


def test_running_example_verdicts(running):
    fx, exp = running
    D, P1 = fx["D"], fx["P1"]
    # threshold 7: infrequent (Section 2.2)
    t7 = int(exp[("P1", "infrequent_at")][0])
    r = O.query(D, P1, t7, 1.0)
    assert r["frequent"] == 0
    # sigma=3, lambda=1: tau=3, infrequent under mIS
    assert O.query(D, P1, 3, 1.0)["frequent"] == 0
    # sigma=2, lambda=1: tau=2; the lexicographic greedy finds Mapping IV: frequent
    assert O.query(D, P1, 2, 1.0)["frequent"] == 1
    # sigma=2, lambda=0.25: tau=1, frequent
    r = O.query(D, P1, 2, 0.25)
    assert r["tau"] == 1 and r["frequent"] == 1
    v = O.query(D, P1, 2, 0.25, mode=O.VERDICT)
    assert v["frequent"] == 1 and v["support"] == 1 and v["embedding_count"] == -1


def test_running_example_p2(running):
    fx, _ = running
    D, P2 = fx["D"], fx["P2"]
    embs = O.brute_embeddings(D, P2)
    cnt, rows = O.enumerate_embeddings(D, P2)
    assert cnt == len(embs) == 4
    assert [tuple(r) for r in rows.tolist()] == embs
    k, sel = O.support_stream(D, P2)
    assert k == 1 and [tuple(r) for r in sel.tolist()] == [(1, 4, 5)]
    assert O.brute_mis(embs) == 1
    assert O.mni(D, P2) == 2


def test_unlabeled_triangle_on_running_graph(running):
    fx, _ = running
    D = relabel_all(fx["D"])
    tri = Pattern(vlabel=[0, 0, 0], edges=[(0, 1), (1, 2), (0, 2)], elabel=[0, 0, 0])
    A = adjacency_matrix(D)
    cnt, _ = O.enumerate_embeddings(D, tri)
    assert cnt == int(np.trace(A @ A @ A)) == 30
    k, sel = O.support_stream(D, tri)
    assert k == 2 and [tuple(r) for r in sel.tolist()] == [(0, 1, 4), (2, 3, 6)]
    assert O.brute_mis(O.brute_embeddings(D, tri)) == 2
    assert O.mni(D, tri) == 7


# ---------------------------------------------------------------------------
# Tightness of Theorem 1 (Section 3.1.1)
# ---------------------------------------------------------------------------

def test_tight_bound_example(tight):
    fx, exp = tight
    Dm, Pm = fx["Dm"], fx["Pm"]
    embs = O.brute_embeddings(Dm, Pm)
    mis = O.brute_mis(embs)
    assert mis == int(exp[("Pm", "mis")][0])
    k, sel = O.support_stream(Dm, Pm)
    # the lexicographic greedy takes the red set: mIS = 1 and M = m * n
    assert k == int(exp[("Pm", "mis_maximal_min")][0])
    assert sorted(sel[0].tolist()) == [int(x) for x in exp[("Pm", "red_set")]]
    assert mis == k * int(exp[("Pm", "n")][0])
    # star closed form: sum_v d(d-1)(d-2) ordered leaf triples; |Aut| = 3! = 6
    d = Dm.degree()
    assert len(embs) == int((d * (d - 1) * (d - 2)).sum()) == 48
    assert len(embs) % automorphisms(Pm) == 0 and automorphisms(Pm) == 6


# ---------------------------------------------------------------------------
# Closed forms on single-label graphs
# ---------------------------------------------------------------------------

def _falling(d, k):
    out = np.ones_like(d)
    for j in range(k):
        out = out * (d - j)
    return out


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_closed_forms_random_graph(seed):
    rng = np.random.default_rng(seed)
    g = relabel_all(tiny_random_graph(rng, 40, 0.15, 1, 1))
    A = adjacency_matrix(g)
    d = g.degree()
    nE = g.num_adj // 2
    tri = Pattern([0, 0, 0], [(0, 1), (1, 2), (0, 2)], [0, 0, 0])
    assert O.count(g, tri, 1 << 40)[0] == int(np.trace(A @ A @ A))
    for k in (1, 2, 3):
        star = Pattern([0] * (k + 1), [(0, j) for j in range(1, k + 1)], [0] * k)
        assert O.count(g, star, 1 << 40)[0] == int(_falling(d, k).sum())
    path = Pattern([0, 0, 0], [(0, 1), (1, 2)], [0, 0])
    assert O.count(g, path, 1 << 40)[0] == int((d * (d - 1)).sum())
    c4 = Pattern([0] * 4, [(0, 1), (1, 2), (2, 3), (3, 0)], [0] * 4)
    A4 = A @ A @ A @ A
    assert O.count(g, c4, 1 << 40)[0] == int(np.trace(A4) - 4 * (d * (d - 1) // 2).sum() - 2 * nE)


def test_labelled_edge_count():
    rng = np.random.default_rng(5)
    g = tiny_random_graph(rng, 60, 0.1, 3, 2)
    el = g.edge_list()
    for a in range(3):
        for b in range(3):
            for e in range(2):
                p = Pattern([a, b], [(0, 1)], [e])
                want = 0
                for u, v, lab in el.tolist():
                    if lab != e:
                        continue
                    lu, lv = int(g.vlabel[u]), int(g.vlabel[v])
                    want += (lu == a and lv == b) + (lu == b and lv == a)
                assert O.count(g, p, 1 << 40)[0] == want


# ---------------------------------------------------------------------------
# Brute force on tiny inputs and the invariants of Section 2.4 / Theorem 1
# ---------------------------------------------------------------------------

def _random_cases(n_cases, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n_cases):
        nv = int(rng.integers(4, 11))
        g = tiny_random_graph(rng, nv, float(rng.uniform(0.2, 0.6)), int(rng.integers(1, 4)),
                              int(rng.integers(1, 3)))
        n = int(rng.integers(2, 5))
        p = random_connected_pattern(rng, n, int(g.vlabel.max()) + 1, int(g.elabel.max()) + 1 if g.num_adj else 1,
                                     extra_edge_p=0.3, prefix_connected=bool(rng.random() < 0.7))
        yield g, p


def test_brute_force_agreement():
    n_nonempty = 0
    for g, p in _random_cases(300, 2024):
        embs = O.brute_embeddings(g, p)
        cnt, rows = O.enumerate_embeddings(g, p)
        assert cnt == len(embs)
        assert [tuple(r) for r in rows.tolist()] == embs
        greedy = O.brute_greedy(embs)
        k2, sel2 = O.support_literal(g, p)
        k3, sel3 = O.support_stream(g, p)
        assert k2 == k3 == len(greedy)
        assert [tuple(r) for r in sel2.tolist()] == greedy == [tuple(r) for r in sel3.tolist()]
        assert O.is_maximal_independent(greedy, embs)
        c, sat, dg = O.count(g, p, 1 << 40)
        assert c == len(embs) and not sat
        assert len(embs) % automorphisms(p) == 0
        if embs:
            n_nonempty += 1
            mis = O.brute_mis(embs)
            # Theorem 1: m <= M <= m n
            assert k3 <= mis <= k3 * p.n
            assert k3 <= O.brute_mni(embs, p.n) == O.mni(g, p)
            assert k3 <= g.num_vertices // p.n
        # verdict mode agrees with the full support at every threshold
        for t in range(1, 5):
            kv, _ = O.support_stream(g, p, stop_at=t)
            assert (kv >= t) == (k3 >= t)
    assert n_nonempty > 100


def test_digest_and_saturation():
    rng = np.random.default_rng(7)
    g = tiny_random_graph(rng, 12, 0.5, 2, 1)
    p = Pattern([0, 1, 0], [(0, 1), (1, 2)], [0, 0])
    embs = O.brute_embeddings(g, p)
    assert len(embs) > 4
    c, sat, dg = O.count(g, p, 1 << 40)
    s1, s2 = 0x243F6A8885A308D3, 0x13198A2E03707344
    want0 = sum(O.tuple_hash(e, s1) for e in embs) % (1 << 64)
    want1 = 0
    for e in embs:
        want1 ^= O.tuple_hash(e, s2)
    assert (c, sat, dg) == (len(embs), False, (want0, want1))
    # the digest depends on the set, not the order
    perm = np.random.default_rng(1).permutation(len(embs))
    assert sum(O.tuple_hash(embs[i], s1) for i in perm) % (1 << 64) == want0
    # saturation: count = min(|M|, cap)
    c2, sat2, _ = O.count(g, p, 3)
    assert c2 == 3 and sat2
    c3, sat3, _ = O.count(g, p, len(embs))
    assert c3 == len(embs) and sat3
    c4, sat4, _ = O.count(g, p, len(embs) + 1)
    assert c4 == len(embs) and not sat4


def test_splitmix64_published_vector():
    # SplitMix64 seeded with 0: the first output is 0xE220A8397B1DCDAF
    # (Vigna's reference generator); tuple_hash of a single 0 applies the
    # same finaliser to seed ^ 0.
    assert O.tuple_hash([0], 0) == 0xE220A8397B1DCDAF


def test_bad_patterns():
    assert not O.pattern_valid(Pattern([0, 0, 0], [(0, 1)], [0]))  # disconnected
    assert not O.pattern_valid(Pattern([0, 0], [(0, 0)], [0]))  # loop
    assert not O.pattern_valid(Pattern([0, 0], [(0, 1), (1, 0)], [0, 0]))  # repeated edge
    assert O.pattern_valid(Pattern([0, 0], [(0, 1)], [0]))


def test_tiny_n_equals_one_and_two():
    rng = np.random.default_rng(3)
    g = tiny_random_graph(rng, 9, 0.4, 2, 1)
    one = Pattern([1], [], [])
    k, _ = O.support_stream(g, one)
    assert k == int((g.vlabel == 1).sum())
    assert math.isclose(O.tau(10, 0.5, 1), 10)


def test_selection_digest():
    # the selected set's digest is the embedding digest's hash over S: where
    # every embedding is selected (a single-vertex pattern, disjoint
    # embeddings) it equals the digest of M; on the running example it is the
    # digest of the two selections under the lexicographic order
    # (Figure 1: (d1, d5, d2) and (d3, d7, d4), 0-based (0, 4, 1) and (2, 6, 3));
    # on random tiny graphs it is the digest of the brute-force greedy
    fx1 = load_fixture("running_example.txt")
    D, P1 = fx1["D"], fx1["P1"]
    one = Pattern([1], [], [])
    r = O.query(D, one, 1, 1.0, O.FULL)
    assert r["support"] == r["embedding_count"] == 3
    assert r["sel_digest"] == r["digest"]
    r = O.query(D, P1, 2, 1.0, O.FULL)
    s1, s2 = 0x243F6A8885A308D3, 0x13198A2E03707344
    sel = [(0, 4, 1), (2, 6, 3)]
    want = (sum(O.tuple_hash(e, s1) for e in sel) % (1 << 64), O.tuple_hash(sel[0], s2) ^ O.tuple_hash(sel[1], s2))
    assert r["sel_digest"] == want
    assert O.query(D, P1, 2, 1.0, O.VERDICT)["sel_digest"] == (0, 0)
    for idx, (g, p) in enumerate(_random_cases(60, 77)):
        greedy = O.brute_greedy(O.brute_embeddings(g, p))
        got = O.query(g, p, 2, 1.0, O.FULL)["sel_digest"]
        assert got == O.rows_digest(np.asarray(greedy, dtype=np.int32).reshape(-1, p.n), p.n), idx


# ---------------------------------------------------------------------------
# Directed graphs (Section 2.2: the problem is stated for labeled, directed
# graphs; a pattern edge (a, b) is a -> b)
# ---------------------------------------------------------------------------

def _directed_cases(n_cases, seed):
    from paper_2404_01585_amd.synth import random_directed_pattern, tiny_random_digraph
    rng = np.random.default_rng(seed)
    for _ in range(n_cases):
        nv = int(rng.integers(3, 10))
        g = tiny_random_digraph(rng, nv, float(rng.uniform(0.15, 0.5)), int(rng.integers(1, 3)),
                                int(rng.integers(1, 3)))
        n = int(rng.integers(2, 5))
        p = random_directed_pattern(rng, n, int(g.vlabel.max()) + 1, int(g.elabel.max()) + 1 if g.num_adj else 1,
                                    prefix_connected=bool(rng.random() < 0.7))
        yield g, p


def test_directed_brute_force_agreement():
    # brute force over all tuples = the literal form = the streaming matcher,
    # in embeddings, the greedy selection and the invariants
    checked = 0
    for g, p in _directed_cases(250, 31):
        G = O.OracleGraph.of(g)
        embs = O.brute_embeddings(g, p)
        cnt, rows = O.enumerate_embeddings(G, p)
        assert cnt == len(embs)
        assert [tuple(int(x) for x in r) for r in rows] == embs
        k_lit, sel_lit = O.support_literal(G, p)
        k_str, sel_str = O.support_stream(G, p)
        greedy = O.brute_greedy(embs)
        assert k_lit == k_str == len(greedy)
        assert [tuple(int(x) for x in r) for r in sel_str] == greedy
        assert O.is_maximal_independent(greedy, embs)
        if embs:
            assert len(greedy) <= O.brute_mis(embs) <= len(greedy) * p.n  # Theorem 1
            assert len(greedy) <= O.brute_mni(embs, p.n)
        checked += len(embs) > 0
    assert checked > 50


def test_directed_closed_forms():
    from paper_2404_01585_amd.synth import tiny_random_digraph
    rng = np.random.default_rng(8)
    for _ in range(5):
        g = tiny_random_digraph(rng, 12, 0.3, 1, 1)
        nv = g.num_vertices
        a = np.zeros((nv, nv), dtype=np.int64)
        src = np.repeat(np.arange(nv), g.degree())
        a[src, g.col] = 1
        out_d, in_d = a.sum(1), a.sum(0)
        recip = (a * a.T).sum(1)
        # directed 3-cycle a -> b -> c -> a: trace(A^3) embeddings
        cyc = Pattern([0, 0, 0], [(0, 1), (1, 2), (2, 0)], [0, 0, 0])
        assert O.count(g, cyc, 1 << 40)[0] == int(np.trace(a @ a @ a))
        # directed 2-path a -> b -> c with a != c
        path = Pattern([0, 0, 0], [(0, 1), (1, 2)], [0, 0])
        assert O.count(g, path, 1 << 40)[0] == int((in_d * out_d - recip).sum())
        # out-star b <- a -> c
        star = Pattern([0, 0, 0], [(0, 1), (0, 2)], [0, 0])
        assert O.count(g, star, 1 << 40)[0] == int((out_d * (out_d - 1)).sum())
        # a reciprocal pair a <-> b
        pair = Pattern([0, 0], [(0, 1), (1, 0)], [0, 0])
        assert O.count(g, pair, 1 << 40)[0] == int(recip.sum())


def test_directed_reduces_to_undirected():
    # an undirected graph given as a directed one (both directions, equal
    # labels) and a pattern whose every edge is reciprocal with equal labels
    # give the undirected embeddings and support
    from paper_2404_01585_amd.synth import csr_from_arcs
    rng = np.random.default_rng(12)
    for _ in range(20):
        g = tiny_random_graph(rng, 9, 0.4, 2, 2)
        src = np.repeat(np.arange(g.num_vertices), g.degree())
        gd = csr_from_arcs(g.num_vertices, src, g.col, g.elabel, g.vlabel)
        p = random_connected_pattern(rng, int(rng.integers(2, 5)), 2, 2)
        pd = Pattern(p.vlabel, [e for a, b in p.edges for e in ((a, b), (b, a))],
                     [l for l in p.elabel for _ in range(2)])
        assert O.query(g, p, 2, 1.0, O.FULL)["support"] == O.query(gd, pd, 2, 1.0, O.FULL)["support"]
        assert O.count(g, p, 1 << 40)[:2] == O.count(gd, pd, 1 << 40)[:2]
