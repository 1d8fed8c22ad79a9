"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer results must match exactly: support, verdict, tau, embedding count,
saturation flag, digest of the embedding set, the selected embeddings in
rank order, and the full embedding list where it is listed."""

import numpy as np
import pytest

from helpers import load_fixture, relabel_all
from oracle import oracle as O
from paper_2404_01585_amd import flexis as fx
from paper_2404_01585_amd.synth import (Graph, Pattern, csr_from_edges, random_connected_pattern, sample_patterns,
                                        tiny_random_graph, workload_graph)

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = fx.Context(device=0)
    yield c


@pytest.fixture(scope="module")
def ctx_small(torch_cuda):
    # tiny slices: every level is cut into many slices with ragged tails; no
    # label-run index, so runs come from binary searches
    c = fx.Context(device=0, slice_rows=64, run_index_bytes=-1)
    yield c


FULL_KEYS = ("tau", "support", "frequent", "embedding_count", "count_saturated", "digest", "sel_digest")


def full_match(dg, g, p, sigma, lam, count_cap=1 << 62, sel=True):
    want = O.query(g, p, sigma, lam, O.FULL, count_cap=count_cap)
    got = dg.support(p, sigma, lam, fx.MODE_FULL, selected_cap=(g.num_vertices if sel else 0))
    for k in FULL_KEYS:
        assert got[k] == want[k], (k, got[k], want[k])
    assert got["status"] == fx.FX_OK and got["exit"] in (fx.EXIT_END, fx.EXIT_EMPTY)
    if sel:
        assert np.array_equal(got["selected"], want["selected"]), (got["selected"], want["selected"])
        # the selection digest is that of the selected rows
        assert got["sel_digest"] == O.rows_digest(got["selected"], p.n)
    return got


def verdict_match(dg, g, p, sigma, lam):
    want = O.query(g, p, sigma, lam, O.VERDICT)
    got = dg.support(p, sigma, lam, fx.MODE_VERDICT)
    for k in ("tau", "support", "frequent", "embedding_count"):
        assert got[k] == want[k], (k, got[k], want[k])


def list_match(dg, g, p, cap=1 << 16):
    cnt_w, rows_w = O.enumerate_embeddings(g, p, cap=cap)
    cnt_g, rows_g = dg.enumerate(p, cap)
    assert cnt_g == cnt_w
    assert np.array_equal(rows_g, rows_w)


# ---------------------------------------------------------------------------

def test_running_example(ctx, ctx_small):
    fx1 = load_fixture("running_example.txt")
    fx2 = load_fixture("tight_bound.txt")
    D, Dm = fx1["D"], fx2["Dm"]
    tri = Pattern([0, 0, 0], [(0, 1), (1, 2), (0, 2)], [0, 0, 0])
    for c in (ctx, ctx_small):
        with c.load_graph(D) as dg:
            for name in ("P1", "P2"):
                _say("running example", name)
                p = fx1[name]
                got = full_match(dg, D, p, 2, 1.0)
                list_match(dg, D, p)
                for sigma, lam in ((3, 1.0), (2, 1.0), (2, 0.25), (7, 1.0)):
                    full_match(dg, D, p, sigma, lam)
                    verdict_match(dg, D, p, sigma, lam)
            assert got["support"] == 1
        Du = relabel_all(D)
        with c.load_graph(Du) as dg:
            _say("unlabeled triangle")
            got = full_match(dg, Du, tri, 2, 1.0)
            assert got["embedding_count"] == 30 and got["support"] == 2
            list_match(dg, Du, tri)
        with c.load_graph(Dm) as dg:
            _say("tight bound example")
            got = full_match(dg, Dm, fx2["Pm"], 1, 1.0)
            assert got["support"] == 1 and got["embedding_count"] == 48
            list_match(dg, Dm, fx2["Pm"])


def mni_match(dg, g, p, sigma):
    """Minimum-image mode against the oracle: the MNI value, its verdict at
    sigma, and the embedding count and digest of FULL mode."""
    want = O.mni(g, p)
    full = O.query(g, p, sigma, 1.0, O.FULL)
    got = dg.support(p, sigma, 1.0, fx.MODE_MNI)
    assert got["support"] == want, (got["support"], want)
    assert got["tau"] == sigma and got["frequent"] == int(want >= max(sigma, 1))
    assert got["embedding_count"] == full["embedding_count"] and got["digest"] == full["digest"]
    assert full["support"] <= want  # the greedy support never exceeds MNI
    return got


def test_mni_mode(ctx, ctx_small, er1k):
    """Minimum-image support (Section 2.4.4): the running example's printed
    value, tiny random graphs (also against brute force), sampled patterns on
    the 1K-vertex graph, alone and as a batch."""
    fx1 = load_fixture("running_example.txt")
    with ctx.load_graph(fx1["D"]) as dg:
        _say("mni running example")
        assert mni_match(dg, fx1["D"], fx1["P1"], 3)["support"] == 3
    for idx, g, p in _tiny_cases(40, seed=404):
        c = ctx if idx % 2 else ctx_small
        with c.load_graph(g) as dg:
            _say("mni tiny", idx, "nv", g.num_vertices, "n", p.n)
            got = mni_match(dg, g, p, 2)
            if p.n <= 4 and g.num_vertices <= 16:
                assert got["support"] == O.brute_mni(O.brute_embeddings(g, p), p.n)
    pats = sample_patterns(er1k, 24, seed=91, kmin=2, kmax=5)
    for c in (ctx, ctx_small):
        with c.load_graph(er1k) as dg:
            alone = []
            for i, p in enumerate(pats):
                _say("mni er1k", i, "n", p.n)
                alone.append(mni_match(dg, er1k, p, 20))
            mix = dg.support_batch(pats, [20] * len(pats), [1.0] * len(pats), fx.MODE_MNI)
            for a, b in zip(alone, mix):
                for k in ("support", "frequent", "embedding_count", "digest", "tau"):
                    assert a[k] == b[k], k


def _tiny_cases(n_cases, seed):
    rng = np.random.default_rng(seed)
    for idx in range(n_cases):
        nv = int(rng.integers(4, 40))
        g = tiny_random_graph(rng, nv, float(rng.uniform(0.08, 0.5)), int(rng.integers(1, 4)), int(rng.integers(1, 3)))
        n = int(rng.integers(1, 6))
        p = random_connected_pattern(rng, n, int(g.vlabel.max()) + 1, int(g.elabel.max()) + 1 if g.num_adj else 1,
                                     extra_edge_p=0.3, prefix_connected=bool(rng.random() < 0.75))
        yield idx, g, p


@pytest.mark.parametrize("which", ["default", "small"])
def test_random_tiny(ctx, ctx_small, which):
    c = ctx if which == "default" else ctx_small
    for idx, g, p in _tiny_cases(150, 99 if which == "default" else 98):
        _say("tiny", which, idx, "nv", g.num_vertices, "n", p.n)
        with c.load_graph(g) as dg:
            full_match(dg, g, p, 2, 1.0)
            list_match(dg, g, p)
            for sigma in (1, 2, 3, 5):
                verdict_match(dg, g, p, sigma, 0.5)


@pytest.fixture(scope="module")
def er1k():
    return workload_graph("er1k")


def test_er1k_sampled_patterns(ctx, ctx_small, er1k):
    g = er1k
    pats = sample_patterns(g, 40, seed=7, kmin=2, kmax=6)
    with ctx.load_graph(g) as dg, ctx_small.load_graph(g) as ds:
        for i, p in enumerate(pats):
            _say("er1k pattern", i, "n", p.n, "m", p.m)
            a = full_match(dg, g, p, 20, 1.0)
            b = full_match(ds, g, p, 20, 1.0)
            assert a["support"] == b["support"]
            verdict_match(dg, g, p, 20, 1.0)
            verdict_match(ds, g, p, 20, 0.3)


def test_capped_slices_and_promotion(ctx_small, er1k):
    """Slices that stop at their row cap (the rest offered again) and stacks
    moved to a larger capacity when few queries are left give the oracle's
    results, alone and in a batch."""
    g = er1k
    pats = sample_patterns(g, 12, seed=77, kmin=4, kmax=7)
    ctx_small.stats(reset=True)
    with ctx_small.load_graph(g) as ds:
        alone = []
        for i, p in enumerate(pats):
            _say("capped slices, pattern", i, "n", p.n, "m", p.m)
            alone.append(full_match(ds, g, p, 20, 1.0))
        mix = ds.support_batch(pats, [20] * len(pats), [1.0] * len(pats), fx.MODE_FULL)
        for a, b in zip(alone, mix):
            for k in ("support", "frequent", "embedding_count", "digest"):
                assert a[k] == b[k], k
    st = ctx_small.stats()
    _say("stats", st)
    assert st["reoffered"] > 0 and st["promotions"] > 0


def test_er1k_listing(ctx, er1k):
    g = er1k
    pats = sample_patterns(g, 6, seed=8, kmin=3, kmax=4)
    with ctx.load_graph(g) as dg:
        for i, p in enumerate(pats):
            _say("er1k listing", i)
            list_match(dg, g, p, cap=1 << 20)


def test_count_cap_saturation(torch_cuda, er1k):
    g = er1k
    star = Pattern([0, 1, 1, 1], [(0, 1), (0, 2), (0, 3)], [0, 0, 0])
    total = O.count(g, star, 1 << 62)[0]
    assert total > 100
    for cap in (1, 7, total // 3, total, total + 1):
        _say("count cap", cap)
        c = fx.Context(device=0, slice_rows=128, count_cap=cap)
        with c.load_graph(g) as dg:
            full_match(dg, g, star, 20, 1.0, count_cap=cap)
        c.close()


def test_symmetric_patterns(ctx, ctx_small):
    # patterns with large automorphism groups (the support phase enumerates
    # one embedding per orbit): stars, paths with equal ends, cycles, cliques,
    # in several vertex numberings, on a graph with two vertex labels
    rng = np.random.default_rng(21)
    g = tiny_random_graph(rng, 300, 0.03, 2, 1)
    pats = [Pattern([0, 0, 0, 0], [(0, 1), (0, 2), (0, 3)], [0] * 3),
            Pattern([0, 0, 0, 0], [(3, 0), (3, 1), (3, 2)], [0] * 3),
            Pattern([1, 0, 0, 1], [(0, 1), (1, 2), (2, 3)], [0] * 3),
            Pattern([0, 1, 0], [(0, 1), (1, 2)], [0] * 2),
            Pattern([0, 0, 0], [(0, 1), (1, 2), (0, 2)], [0] * 3),
            Pattern([0, 0, 0, 0], [(0, 1), (1, 2), (2, 3), (3, 0)], [0] * 4),
            Pattern([0, 0, 0, 0], [(0, 2), (2, 1), (1, 3), (3, 0)], [0] * 4),
            Pattern([0, 0, 0, 0], [(a, b) for a in range(4) for b in range(a + 1, 4)], [0] * 6),
            Pattern([0, 0, 1, 0, 0], [(2, 0), (2, 1), (2, 3), (2, 4)], [0] * 4)]
    for which, c in (("default", ctx), ("small", ctx_small)):
        with c.load_graph(g) as dg:
            for i, p in enumerate(pats):
                _say("symmetric", which, i)
                full_match(dg, g, p, 2, 1.0)
                for sigma in (1, 5, 40):
                    verdict_match(dg, g, p, sigma, 0.5)
            got = dg.support_batch(pats, [3] * len(pats), [1.0] * len(pats), fx.MODE_FULL)
            for p, r in zip(pats, got):
                want = O.query(g, p, 3, 1.0, O.FULL)
                for k in ("support", "frequent", "embedding_count", "digest"):
                    assert r[k] == want[k], (k, r[k], want[k])


@pytest.mark.timeout(300)
def test_wide_patterns_on_hubs(torch_cuda):
    # 5- to 13-vertex patterns (every register width of a partial row: up to
    # 4, 8 and 16 vertices) on a small power-law graph whose hubs have label
    # runs long enough for the binary searches; the count is capped so the
    # enumeration stays small, the support is exact
    from paper_2404_01585_amd.synth import chung_lu
    g = chung_lu(3000, 9000, 2.1, 11, 4, None, 2)
    pats = (sample_patterns(g, 6, seed=4, kmin=5, kmax=8, shapes=("cycle", "chord", "tree"))
            + sample_patterns(g, 12, seed=5, kmin=9, kmax=13, shapes=("cycle", "chord", "tree")))
    cap = 1 << 20
    for which, c in (("index", fx.Context(device=0, count_cap=cap)),
                     ("search", fx.Context(device=0, count_cap=cap, slice_rows=256, run_index_bytes=-1))):
        with c.load_graph(g) as dg:
            for i, p in enumerate(pats):
                _say("wide", which, i, "n", p.n)
                full_match(dg, g, p, 2, 1.0, count_cap=cap)
                verdict_match(dg, g, p, 5, 0.5)
        c.close()


def test_edge_cases(ctx):
    # isolated vertices, an empty adjacency, single-vertex patterns, absent labels
    g = csr_from_edges(6, [0, 1], [1, 2], [0, 0], [0, 0, 1, 1, 2, 2])
    single = Pattern([1], [], [])
    absent = Pattern([0, 9], [(0, 1)], [0])
    absent_el = Pattern([0, 0], [(0, 1)], [5])
    with ctx.load_graph(g) as dg:
        _say("edge cases")
        got = full_match(dg, g, single, 1, 1.0)
        assert got["support"] == 2
        for p in (absent, absent_el):
            r = dg.support(p, 1, 1.0, fx.MODE_FULL)
            assert r["support"] == 0 and r["embedding_count"] == 0 and r["frequent"] == 0
            assert dg.support(p, 1, 1.0, fx.MODE_VERDICT)["frequent"] == 0
    empty = csr_from_edges(5, [], [], [], [0, 0, 0, 1, 1])
    with ctx.load_graph(empty) as dg:
        full_match(dg, empty, Pattern([0], [], []), 3, 1.0)
        full_match(dg, empty, Pattern([0, 0], [(0, 1)], [0]), 1, 1.0)
    # the largest pattern: a 16-vertex path in a 40-vertex path graph
    chain = csr_from_edges(40, list(range(39)), list(range(1, 40)), [0] * 39, [0] * 40)
    path16 = Pattern([0] * 16, [(i, i + 1) for i in range(15)], [0] * 15)
    with ctx.load_graph(chain) as dg:
        _say("path16")
        got = full_match(dg, chain, path16, 2, 1.0)
        assert got["embedding_count"] == 2 * (40 - 15)
        list_match(dg, chain, path16)


def test_errors(ctx):
    bad = Graph(row_ptr=np.array([0, 1, 1], dtype=np.int64), col=np.array([1], dtype=np.int32),
                vlabel=np.array([0, 0], dtype=np.int32), elabel=np.array([0], dtype=np.int32))
    with pytest.raises(fx.FxError) as e:
        ctx.load_graph(bad)
    assert e.value.status == fx.FX_EGRAPH
    g = csr_from_edges(4, [0, 1, 2], [1, 2, 3], [0, 0, 0], [0, 0, 0, 0])
    with ctx.load_graph(g) as dg:
        with pytest.raises(fx.FxError) as e:
            dg.support(Pattern([0, 0, 0], [(0, 1)], [0]), 1, 1.0)
        assert e.value.status == fx.FX_EPATTERN
        with pytest.raises(fx.FxError) as e:
            dg.support(Pattern([0] * 17, [(i, i + 1) for i in range(16)], [0] * 16), 1, 1.0)
        assert e.value.status == fx.FX_ELIMIT
        with pytest.raises(fx.FxError) as e:
            dg.support(Pattern([0, 0], [(0, 1)], [0]), 0, 1.0)
        assert e.value.status == fx.FX_EINVAL
        with pytest.raises(fx.FxError) as e:
            dg.support(Pattern([0, 0], [(0, 1)], [0]), 1, 1.5)
        assert e.value.status == fx.FX_EINVAL


def test_device_resident_input(ctx, er1k):
    import torch
    g = er1k
    gd = Graph(row_ptr=torch.from_numpy(g.row_ptr).cuda(), col=torch.from_numpy(g.col).cuda(),
               vlabel=torch.from_numpy(g.vlabel).cuda(), elabel=torch.from_numpy(g.elabel).cuda())
    p = Pattern([0, 1, 2], [(0, 1), (1, 2)], [0, 0])
    _say("device resident graph")
    with ctx.load_graph(gd, on_device=True) as dg:
        full_match(dg, g, p, 20, 1.0)


def _mining_candidates(g, sigma, lam, levels):
    from paper_2404_01585_amd import mining

    def ev(ps, s, l):
        return [O.query(g, p, s, l, mode=O.VERDICT) for p in ps]

    r = mining.mine(g, sigma, lam, levels, ev, tau_fn=O.tau)
    return [p for lvl in r["levels"] for p in lvl]


def test_merge_generator_mining(ctx, er1k):
    """Algorithm 1 with the merge generator (levels by vertex count, up to 4
    vertices) gives the same candidates and verdicts with the device's
    verdicts as with the oracle's."""
    from paper_2404_01585_amd import generate

    g = er1k

    def ev_oracle(ps, s, l):
        return [O.query(g, p, s, l, mode=O.VERDICT) for p in ps]

    want = generate.mine_by_vertices(g, 20, 1.0, 4, ev_oracle, O.tau)
    with ctx.load_graph(g) as dg:
        def ev_dev(ps, s, l):
            return dg.support_batch(ps, [s] * len(ps), [l] * len(ps), fx.MODE_VERDICT)

        got = generate.mine_by_vertices(g, 20, 1.0, 4, ev_dev, fx.tau)
    assert len(got["levels"]) == len(want["levels"])
    for lv, (a, b) in enumerate(zip(got["levels"], want["levels"])):
        _say("merge mining level", lv, len(a))
        assert [(p.vlabel, p.edges, p.elabel) for p in a] == [(p.vlabel, p.edges, p.elabel) for p in b]
        assert [r["frequent"] for r in got["results"][lv]] == [r["frequent"] for r in want["results"][lv]]


def test_er1k_mining_batch(ctx, er1k):
    """Every candidate of the mining levels up to 4 edges on the 1K-vertex
    graph (sigma 20), as one batch, FULL and VERDICT, against the oracle
    pattern by pattern: support, verdict, count, embedding digest and the
    selected set's digest."""
    g = er1k
    cands = _mining_candidates(g, 20, 1.0, 4)
    assert len(cands) > 4000 and max(p.m for p in cands) == 4
    with ctx.load_graph(g) as dg:
        for lam in (1.0, 0.3):
            _say("er1k batch FULL lambda", lam, "patterns", len(cands))
            got = dg.support_batch(cands, [20] * len(cands), [lam] * len(cands), fx.MODE_FULL)
            for p, r in zip(cands, got):
                want = O.query(g, p, 20, lam, O.FULL)
                for k in FULL_KEYS:
                    assert r[k] == want[k], (p, k, r[k], want[k])
            _say("er1k batch VERDICT lambda", lam)
            got = dg.support_batch(cands, [20] * len(cands), [lam] * len(cands), fx.MODE_VERDICT)
            for p, r in zip(cands, got):
                want = O.query(g, p, 20, lam, O.VERDICT)
                for k in ("tau", "support", "frequent", "embedding_count"):
                    assert r[k] == want[k], (p, k, r[k], want[k])


def test_alone_equals_in_the_mix(ctx, ctx_small, er1k):
    """A pattern's result does not depend on what else is in the batch, on the
    batch order, or on the slice capacity (tolerance 0: all results are integers)."""
    g = er1k
    pats = sample_patterns(g, 60, seed=31, kmin=2, kmax=5)
    rng = np.random.default_rng(5)
    with ctx.load_graph(g) as dg, ctx_small.load_graph(g) as ds:
        alone = [dg.support(p, 20, 0.5, fx.MODE_FULL) for p in pats]
        mix = dg.support_batch(pats, [20] * len(pats), [0.5] * len(pats), fx.MODE_FULL)
        perm = rng.permutation(len(pats))
        mix2 = ds.support_batch([pats[i] for i in perm], [20] * len(pats), [0.5] * len(pats), fx.MODE_FULL)
        keys = ("tau", "support", "frequent", "embedding_count", "count_saturated", "digest")
        for i in range(len(pats)):
            _say("mix", i)
            for k in keys:
                assert alone[i][k] == mix[i][k], (i, k)
        for j, i in enumerate(perm):
            for k in keys:
                assert alone[i][k] == mix2[j][k], (i, k)


@pytest.mark.parametrize("slice_rows", [0, 64])
def test_no_digest_counts(torch_cuda, er1k, slice_rows):
    """Without the digest, counts of leaf-ended patterns come from the closed
    form (run length minus matched vertices in the run); they must equal the
    oracle's enumeration exactly, as must support and verdict."""
    g = er1k
    cands = _mining_candidates(g, 20, 1.0, 3) + sample_patterns(g, 40, seed=17, kmin=2, kmax=6)
    c = fx.Context(device=0, slice_rows=slice_rows, no_digest=True, run_index_bytes=(-1 if slice_rows else 0))
    with c.load_graph(g) as dg:
        _say("no digest, slice rows", slice_rows, "patterns", len(cands))
        got = dg.support_batch(cands, [20] * len(cands), [0.5] * len(cands), fx.MODE_FULL)
        for p, r in zip(cands, got):
            want = O.query(g, p, 20, 0.5, O.FULL)
            for k in ("tau", "support", "frequent", "embedding_count", "count_saturated"):
                assert r[k] == want[k], (p, k, r[k], want[k])
            assert r["digest"] == (0, 0)
    # tiny graphs, including labels that collide with earlier pattern vertices
    for idx, gg, p in _tiny_cases(80, 555):
        with c.load_graph(gg) as dg:
            want = O.query(gg, p, 2, 1.0, O.FULL)
            r = dg.support(p, 2, 1.0, fx.MODE_FULL)
            for k in ("support", "embedding_count"):
                assert r[k] == want[k], (idx, k, r[k], want[k])
    c.close()


def test_server_alone_equals_in_the_mix(ctx, er1k):
    """Queries submitted concurrently from several threads to the
    continuous-batching server get exactly the results fx_support gives them
    alone (tolerance 0)."""
    import threading
    import time

    g = er1k
    pats = sample_patterns(g, 120, seed=41, kmin=2, kmax=6)
    rng = np.random.default_rng(9)
    sig = [int(x) for x in rng.integers(5, 60, size=len(pats))]
    lam = [float(x) for x in rng.choice([0.1, 0.5, 1.0], size=len(pats))]
    modes = [int(x) for x in rng.integers(0, 2, size=len(pats))]
    with ctx.load_graph(g) as dg:
        alone = [dg.support(p, s, l, m) for p, s, l, m in zip(pats, sig, lam, modes)]
        # every query alone is the oracle's answer
        for p, sg, lm, md, a in zip(pats, sig, lam, modes, alone):
            want = O.query(g, p, sg, lm, md)
            for k in (("tau", "support", "frequent", "embedding_count") +
                      (("count_saturated", "digest", "sel_digest") if md == fx.MODE_FULL else ())):
                assert a[k] == want[k], (k, a[k], want[k])
        with fx.Server(dg, max_active=32, step_candidates=1 << 16) as srv:
            tickets = [None] * len(pats)

            def submitter(idx):
                for i in idx:
                    tickets[i] = srv.submit(pats[i], sig[i], lam[i], modes[i])
                    time.sleep(float(rng.random()) * 1e-3)

            parts = [list(range(k, len(pats), 4)) for k in range(4)]
            th = [threading.Thread(target=submitter, args=(pp,)) for pp in parts]
            for t in th:
                t.start()
            for t in th:
                t.join()
            _say("server: all submitted")
            got = [srv.wait(t, 60_000_000) for t in tickets]
            st = srv.stats()
        assert st["queries"] > 0
        for i in range(len(pats)):
            for k in ("tau", "support", "frequent", "embedding_count", "count_saturated", "digest", "sel_digest",
                      "exit"):
                assert got[i][k] == alone[i][k], (i, k, got[i][k], alone[i][k])
            assert got[i]["device_ms"] >= 0 and got[i]["status"] == fx.FX_OK
        # errors are reported at submission; unknown tickets are rejected; the
        # graph cannot go while a server holds it
        with fx.Server(dg) as srv:
            with pytest.raises(fx.FxError) as e:
                srv.submit(pats[0], 0, 1.0)
            assert e.value.status == fx.FX_EINVAL
            with pytest.raises(fx.FxError) as e:
                srv.submit(Pattern([0, 0, 0], [(0, 1)], [0]), 1, 1.0)
            assert e.value.status == fx.FX_EPATTERN
            with pytest.raises(fx.FxError):
                srv.poll(123456)
            with pytest.raises(fx.FxError) as e:
                dg.close()
            assert e.value.status == fx.FX_EBUSY
            t = srv.submit(pats[1], 20, 1.0)
            r = srv.wait(t)
            assert r["support"] == alone[1]["support"] or modes[1] != fx.MODE_FULL


def test_autotune_keeps_results(torch_cuda, er1k, tmp_path):
    """The autotuner picks a launch shape by timing; results never change, and
    a second call with the same cache file applies the cached choice."""
    g = er1k
    cands = _mining_candidates(g, 20, 1.0, 2)
    c = fx.Context(device=0)
    with c.load_graph(g) as dg:
        batch = fx.PatternBatch(cands)
        cache = str(tmp_path / "tune.txt")
        _say("autotune")
        t1 = dg.autotune(batch, 20, 1.0, fx.MODE_FULL, cache_path=cache)
        assert t1["from_cache"] == 0 and t1["trials"] >= 10
        assert t1["items_per_thread"] in (2, 4, 8)
        got = dg.support_batch(cands, [20] * len(cands), [1.0] * len(cands), fx.MODE_FULL)
        for p, r in zip(cands, got):
            want = O.query(g, p, 20, 1.0, O.FULL)
            for k in ("support", "frequent", "embedding_count", "digest"):
                assert r[k] == want[k], (p, k)
        t2 = dg.autotune(batch, 20, 1.0, fx.MODE_FULL, cache_path=cache)
        assert t2["from_cache"] == 1
        for k in ("slice_rows", "step_candidates", "items_per_thread", "last_span_init", "lanes", "max_active"):
            assert t2[k] == t1[k]
        assert t1["lanes"] in (1, 2, 3)
    c.close()


def test_launch_shapes_agree(torch_cuda, er1k, tmp_path):
    """Every launch shape the tuner may pick (candidates per thread, one to
    three pipeline lanes, small slices and greedy slices) gives the same
    results; each shape is applied through a tuning-cache entry."""
    g = er1k
    cands = _mining_candidates(g, 20, 1.0, 2)
    batch = fx.PatternBatch(cands)
    ref = None
    for items, lanes, slice_rows, last in ((2, 1, 1 << 15, 1024), (8, 2, 1 << 15, 16384), (4, 1, 1 << 17, 4096),
                                           (4, 3, 1 << 15, 4096)):
        c = fx.Context(device=0)
        with c.load_graph(g) as dg:
            cache = str(tmp_path / f"shape_{items}_{lanes}.txt")
            dg.autotune(batch, 20, 1.0, fx.MODE_FULL, cache_path=cache)  # writes the key
            key = open(cache).read().split()[0]
            with open(cache, "w") as f:
                f.write(f"{key} {slice_rows} {1 << 22} {items} {last} {lanes} {64 if lanes == 1 else 4096} 1.0\n")
            t = dg.autotune(batch, 20, 1.0, fx.MODE_FULL, cache_path=cache)
            assert t["from_cache"] == 1 and t["lanes"] == lanes and t["items_per_thread"] == items
            _say("shape", items, lanes, slice_rows, last)
            got = dg.support_batch(cands, [20] * len(cands), [1.0] * len(cands), fx.MODE_FULL)
            ver = dg.support_batch(cands, [20] * len(cands), [0.5] * len(cands), fx.MODE_VERDICT)
        c.close()
        row = [(r["support"], r["frequent"], r["embedding_count"], tuple(r["digest"])) for r in got]
        row += [(r["support"], r["frequent"]) for r in ver]
        if ref is None:
            ref = row
            for p, r in zip(cands, got):
                want = O.query(g, p, 20, 1.0, O.FULL)
                for k in ("support", "frequent", "embedding_count", "digest"):
                    assert r[k] == want[k], (p, k)
        assert row == ref


def test_verdict_bound_exit(torch_cuda, er1k):
    """VERDICT queries whose support can no longer reach tau stop early
    (one selection per root not yet finished, Section 3.2.2, and at most the
    disjointness bound of Section 3.1.2): the verdicts equal the oracle's, and
    the exit fires.  Thresholds sit near the disjointness bound so that few
    roots are left when it is decided; small slices give many steps."""
    g = er1k
    pats = sample_patterns(g, 30, seed=123, kmin=2, kmax=5)
    nlab = np.bincount(g.vlabel)
    cases = []
    for p in pats:
        cnt = np.bincount(np.asarray(p.vlabel), minlength=nlab.shape[0])
        ub = min(g.num_vertices // p.n, min(int(nlab[l]) // int(c) for l, c in enumerate(cnt) if c))
        for frac in (1.0, 0.9, 0.75, 0.5):
            cases.append((p, max(1, int(ub * frac))))
    c = fx.Context(device=0, slice_rows=64, run_index_bytes=-1)
    with c.load_graph(g) as dg:
        for lanes in (1, 2):
            c.set("lanes", lanes)
            c.stats(reset=True)
            _say("bound exit, lanes", lanes, "cases", len(cases))
            got = dg.support_batch([p for p, _ in cases], [s for _, s in cases], [1.0] * len(cases),
                                   fx.MODE_VERDICT)
            alone = [dg.support(p, s, 1.0, fx.MODE_VERDICT) for p, s in cases[:40]]
            st = c.stats()
            _say("stats", st)
            for (p, sg), r in zip(cases, got):
                want = O.query(g, p, sg, 1.0, O.VERDICT)
                for k in ("tau", "support", "frequent", "embedding_count"):
                    assert r[k] == want[k], (p, sg, k, r[k], want[k])
                if r["exit"] == fx.EXIT_BOUND:
                    assert r["frequent"] == 0
                if r["exit"] == fx.EXIT_REACHED:
                    assert r["frequent"] == 1
            for a, b in zip(alone, got):
                assert (a["frequent"], a["support"]) == (b["frequent"], b["support"])
            assert st["exits_bound"] > 0
            assert sum(r["exit"] == fx.EXIT_BOUND for r in got) > 0
    c.close()


def test_lone_growth_fires(torch_cuda, er1k):
    """The stacks of VERDICT queries counted as left nearly alone grow where
    the used-set rule would keep them (here every query counts as alone from
    its first step), and the verdicts stay the oracle's."""
    g = er1k
    pats = sample_patterns(g, 16, seed=321, kmin=4, kmax=7)
    c = fx.Context(device=0, slice_rows=64, run_index_bytes=-1)
    c.set("promote_after", 0)
    c.set("lone_after", 0)
    c.set("lone_queries", 1 << 20)
    assert c.get("lone_after") == 0
    with c.load_graph(g) as dg:
        c.stats(reset=True)
        for sg in (20, 60):
            _say("lone growth sigma", sg)
            got = dg.support_batch(pats, [sg] * len(pats), [1.0] * len(pats), fx.MODE_VERDICT)
            for p, r in zip(pats, got):
                want = O.query(g, p, sg, 1.0, O.VERDICT)
                for k in ("tau", "support", "frequent"):
                    assert r[k] == want[k], (p, k, r[k], want[k])
        st = c.stats()
        _say("stats", st)
        assert st["lone_promotions"] > 0
    c.close()


@pytest.mark.parametrize("chain_steps", [1, 3, 16])
def test_device_scheduled_chains(torch_cuda, er1k, chain_steps):
    """Queries whose steps are scheduled on the device (a captured chain of
    steps replayed with host work between the replays) give the oracle's
    results, alone (a batch of one) and in a batch, in every mode; small
    slices make every query run many steps across many chains."""
    g = er1k
    pats = sample_patterns(g, 24, seed=808, kmin=2, kmax=6)
    c = fx.Context(device=0, slice_rows=64, run_index_bytes=-1)
    c.set("chain_queries", 64)
    c.set("chain_steps", chain_steps)
    with c.load_graph(g) as dg:
        c.stats(reset=True)
        for i, p in enumerate(pats[:8]):
            _say("chain alone", chain_steps, i, "n", p.n)
            r = dg.support_batch([p], [20], [1.0], fx.MODE_FULL)[0]
            want = O.query(g, p, 20, 1.0, O.FULL)
            for k in FULL_KEYS:
                assert r[k] == want[k], (k, r[k], want[k])
            r = dg.support_batch([p], [20], [0.5], fx.MODE_VERDICT)[0]
            want = O.query(g, p, 20, 0.5, O.VERDICT)
            for k in ("tau", "support", "frequent"):
                assert r[k] == want[k], (k, r[k], want[k])
        st = c.stats(reset=True)
        _say("stats alone", st)
        assert st["chains"] > 0 and st["chain_steps"] > 0
        for lam in (1.0, 0.3):
            _say("chain batch FULL", chain_steps, lam)
            got = dg.support_batch(pats, [20] * len(pats), [lam] * len(pats), fx.MODE_FULL)
            for p, r in zip(pats, got):
                want = O.query(g, p, 20, lam, O.FULL)
                for k in FULL_KEYS:
                    assert r[k] == want[k], (p, k, r[k], want[k])
            got = dg.support_batch(pats, [20] * len(pats), [lam] * len(pats), fx.MODE_VERDICT)
            for p, r in zip(pats, got):
                want = O.query(g, p, 20, lam, O.VERDICT)
                for k in ("tau", "support", "frequent", "embedding_count"):
                    assert r[k] == want[k], (p, k, r[k], want[k])
        got = dg.support_batch(pats, [20] * len(pats), [1.0] * len(pats), fx.MODE_MNI)
        for p, r in zip(pats, got):
            assert r["support"] == O.mni(g, p)
        st = c.stats()
        _say("stats batch", st)
        assert st["chains"] > 0
        # the same batch with every step scheduled on the host
        c.set("chain_queries", 0)
        ref = dg.support_batch(pats, [20] * len(pats), [1.0] * len(pats), fx.MODE_FULL)
        c.set("chain_queries", 64)
        again = dg.support_batch(pats, [20] * len(pats), [1.0] * len(pats), fx.MODE_FULL)
        for a, b in zip(ref, again):
            for k in FULL_KEYS + ("exit",):
                assert a[k] == b[k], k
    c.close()


def test_step_checks_on_real_steps(torch_cuda, er1k):
    """With check_steps on, every host-scheduled step's segment table and the
    tile map the device built are checked against the buffers sized for them
    (small slices: ragged tails, capped slices, promotions); no check fires
    and the results stay the oracle's."""
    g = er1k
    pats = sample_patterns(g, 20, seed=909, kmin=2, kmax=7)
    c = fx.Context(device=0, slice_rows=64, run_index_bytes=-1)
    c.set("check_steps", 1)
    with c.load_graph(g) as dg:
        for mode, om in ((fx.MODE_FULL, O.FULL), (fx.MODE_VERDICT, O.VERDICT)):
            _say("step checks mode", mode)
            got = dg.support_batch(pats, [20] * len(pats), [0.5] * len(pats), mode)
            for p, r in zip(pats, got):
                want = O.query(g, p, 20, 0.5, om)
                for k in ("tau", "support", "frequent", "embedding_count"):
                    assert r[k] == want[k], (p, k, r[k], want[k])
        for p in pats[:4]:
            list_match(dg, g, p)
    c.close()


def test_exact_mis_mode(ctx, ctx_small):
    """Exact maximum independent set (Section 2.4.2) as a support mode: the
    paper's printed values (the running example's P1: 2; the tightness example
    of Theorem 1: 4), brute force over all independent sets on tiny graphs,
    and Theorem 1's bounds around the greedy support (m <= M <= m n)."""
    fx1 = load_fixture("running_example.txt")
    fx2 = load_fixture("tight_bound.txt")
    with ctx.load_graph(fx1["D"]) as dg:
        r = dg.support(fx1["P1"], 2, 1.0, fx.MODE_MIS)
        assert r["support"] == 2 and r["embedding_count"] == 6 and r["tau"] == 2 and r["frequent"] == 1
        assert dg.support(fx1["P1"], 3, 1.0, fx.MODE_MIS)["frequent"] == 0
    with ctx.load_graph(fx2["Dm"]) as dg:
        r = dg.support(fx2["Pm"], 1, 1.0, fx.MODE_MIS)
        assert r["support"] == 4 and r["embedding_count"] == 48
        greedy = dg.support(fx2["Pm"], 1, 1.0, fx.MODE_FULL)["support"]
        assert greedy == 1  # the bound m <= M <= m n is tight here: M = n m
    n_checked = 0
    for idx, g, p in _tiny_cases(60, seed=606):
        c = ctx if idx % 2 else ctx_small
        with c.load_graph(g) as dg:
            embs = O.brute_embeddings(g, p) if g.num_vertices <= 16 and p.n <= 4 else None
            full = O.query(g, p, 2, 1.0, O.FULL)
            if full["embedding_count"] > 4096:  # beyond the exact mode's size limit
                with pytest.raises(fx.FxError) as e:
                    dg.support(p, 2, 1.0, fx.MODE_MIS)
                assert e.value.status == fx.FX_ELIMIT
                continue
            _, rows = O.enumerate_embeddings(g, p, cap=4096)
            if len({frozenset(int(v) for v in row) for row in rows}) > 256:  # beyond the distinct-set limit
                with pytest.raises(fx.FxError) as e:
                    dg.support(p, 2, 1.0, fx.MODE_MIS)
                assert e.value.status == fx.FX_ELIMIT
                continue
            r = dg.support(p, 2, 1.0, fx.MODE_MIS)
            _say("mis tiny", idx, "nv", g.num_vertices, "n", p.n, "mis", r["support"])
            assert r["embedding_count"] == full["embedding_count"]
            m = full["support"]
            assert m <= r["support"] <= m * p.n  # Theorem 1
            if embs is not None:
                assert r["support"] == O.brute_mis(embs)
                n_checked += 1
    assert n_checked >= 10
    # a batch gives the same values; too large an instance is refused
    g = csr_from_edges(12, list(range(11)), list(range(1, 12)), [0] * 11, [0] * 12)
    pats = [Pattern([0, 0], [(0, 1)], [0]), Pattern([0, 0, 0], [(0, 1), (1, 2)], [0, 0])]
    with ctx.load_graph(g) as dg:
        got = dg.support_batch(pats, [1, 1], [1.0, 1.0], fx.MODE_MIS)
        assert [r["support"] for r in got] == [6, 4]  # a 12-vertex path: 6 disjoint edges, 4 disjoint 3-paths
    def complete(k):
        e = [(a, b) for a in range(k) for b in range(a + 1, k)]
        return csr_from_edges(k, [a for a, _ in e], [b for _, b in e], [0] * len(e), [0] * k)

    with ctx.load_graph(complete(20)) as dg:  # 20 * 19 * 18 embeddings of a 3-path: more than 4096
        with pytest.raises(fx.FxError) as e:
            dg.support(Pattern([0, 0, 0], [(0, 1), (1, 2)], [0, 0]), 1, 1.0, fx.MODE_MIS)
        assert e.value.status == fx.FX_ELIMIT
    with ctx.load_graph(complete(30)) as dg:  # 435 distinct edges: more than 256 vertex sets
        with pytest.raises(fx.FxError) as e:
            dg.support(Pattern([0, 0], [(0, 1)], [0]), 1, 1.0, fx.MODE_MIS)
        assert e.value.status == fx.FX_ELIMIT
        assert dg.support(Pattern([0, 0], [(0, 1)], [0]), 1, 1.0, fx.MODE_FULL)["support"] == 15


def test_exact_mis_across_stack_growth(torch_cuda):
    """Exact MIS of a query whose stack grows while it enumerates (the
    embeddings collected so far move with it): 3-vertex paths in a 30-vertex
    path among 300 isolated vertices (many roots, few embeddings); a path of
    k vertices holds floor(k / 3) disjoint 3-paths."""
    nv = 330
    g = csr_from_edges(nv, list(range(29)), list(range(1, 30)), [0] * 29, [0] * nv)
    p = Pattern([0, 0, 0], [(0, 1), (1, 2)], [0, 0])
    c = fx.Context(device=0, slice_rows=64, run_index_bytes=-1)
    c.set("promote_after", 1)
    with c.load_graph(g) as dg:
        c.stats(reset=True)
        r = dg.support(p, 1, 1.0, fx.MODE_MIS)
        st = c.stats()
        _say("mis growth", r, st["promotions"])
        assert r["support"] == 10 and r["embedding_count"] == 2 * 28
        assert st["promotions"] > 0
    c.close()


def test_directed_graphs(ctx, ctx_small):
    """Directed data graphs and patterns (Section 2.2): a pattern edge (a, b)
    maps onto a data edge f(a) -> f(b); reciprocal pairs carry their own
    labels.  Every field against the oracle (selected embeddings, listings,
    VERDICT, MNI, exact MIS) on tiny random digraphs, then a batch on a
    1,000-vertex random digraph."""
    from paper_2404_01585_amd.synth import random_directed_pattern, tiny_random_digraph
    rng = np.random.default_rng(1234)
    for idx in range(80):
        nv = int(rng.integers(4, 30))
        g = tiny_random_digraph(rng, nv, float(rng.uniform(0.05, 0.4)), int(rng.integers(1, 3)),
                                int(rng.integers(1, 3)))
        p = random_directed_pattern(rng, int(rng.integers(2, 6)), int(g.vlabel.max()) + 1,
                                    int(g.elabel.max()) + 1 if g.num_adj else 1,
                                    prefix_connected=bool(rng.random() < 0.75))
        c = ctx if idx % 2 else ctx_small
        _say("directed tiny", idx, "nv", nv, "n", p.n, "m", p.m)
        with c.load_graph(g) as dg:
            full_match(dg, g, p, 2, 1.0)
            list_match(dg, g, p)
            for sigma in (1, 3):
                verdict_match(dg, g, p, sigma, 0.5)
            assert dg.support(p, 2, 1.0, fx.MODE_MNI)["support"] == O.mni(g, p)
            cnt, rows = O.enumerate_embeddings(g, p, cap=4096)
            if cnt <= 4096 and len({frozenset(int(v) for v in r) for r in rows}) <= 64:
                mis = dg.support(p, 1, 1.0, fx.MODE_MIS)["support"]
                assert mis == O.brute_mis([tuple(int(v) for v in r) for r in rows])
    # a larger random digraph, one batch
    gb = tiny_random_digraph(rng, 1000, 0.008, 4, 2)
    pats = [random_directed_pattern(rng, int(rng.integers(2, 5)), 4, 2) for _ in range(40)]
    with ctx.load_graph(gb) as dg:
        _say("directed batch", len(pats))
        got = dg.support_batch(pats, [5] * len(pats), [0.5] * len(pats), fx.MODE_FULL)
        for p, r in zip(pats, got):
            want = O.query(gb, p, 5, 0.5, O.FULL)
            for k in FULL_KEYS:
                assert r[k] == want[k], (p, k, r[k], want[k])
    # errors: a repeated arc; a directed graph with a self-loop
    with ctx.load_graph(gb) as dg:
        with pytest.raises(fx.FxError) as e:
            dg.support(Pattern([0, 0], [(0, 1), (0, 1)], [0, 0]), 1, 1.0)
        assert e.value.status == fx.FX_EPATTERN
        r = dg.support(Pattern([0, 0], [(0, 1), (1, 0)], [0, 0]), 1, 1.0)  # a reciprocal pair is fine
        assert r["embedding_count"] == O.query(gb, Pattern([0, 0], [(0, 1), (1, 0)], [0, 0]), 1, 1.0)["embedding_count"]
    from paper_2404_01585_amd.synth import csr_from_arcs
    bad = csr_from_arcs(3, [0, 1], [0, 2], [0, 0], [0, 0, 0])
    with pytest.raises(fx.FxError) as e:
        ctx.load_graph(bad)
    assert e.value.status == fx.FX_EGRAPH


def test_both_expansion_forms(torch_cuda, er1k):
    """The single-pass expansion (one kernel per step, positions by look-back;
    the default for steps of at most 64 workgroups) and the multi-kernel form
    (probe, block scans, scatter, offset fix-up; the default for larger steps)
    each give the oracle's results when every step takes it: tiny graphs with 64-row slices (every
    level cut at its row cap many times), a mining batch, and device-scheduled
    chains; the launch counts show which form ran."""
    g = er1k
    cands = _mining_candidates(g, 20, 1.0, 3)
    pats = sample_patterns(g, 12, seed=909, kmin=2, kmax=6)
    for fused in (1, 0):
        small = fx.Context(device=0, slice_rows=64, run_index_bytes=-1)
        small.set("fused", fused)
        small.set("fused_below", 0)  # every step in the form under test (small steps default to the single pass)
        assert small.get("fused") == fused and small.get("fused_below") == 0
        small.stats(reset=True)
        for idx, gt, p in _tiny_cases(40, 97):
            _say("forms fused", fused, "tiny", idx)
            with small.load_graph(gt) as dg:
                full_match(dg, gt, p, 2, 1.0)
                list_match(dg, gt, p)
                verdict_match(dg, gt, p, 3, 0.5)
        st = small.stats(reset=True)
        assert st["probe_launches"] > 0
        assert (st["scatter_launches"] == 0) if fused else (st["scatter_launches"] == st["probe_launches"])
        big = fx.Context(device=0)
        big.set("fused", fused)
        big.set("fused_below", 0)
        with big.load_graph(g) as dg:
            _say("forms fused", fused, "batch", len(cands))
            got = dg.support_batch(cands, [20] * len(cands), [1.0] * len(cands), fx.MODE_FULL)
            for p, r in zip(cands, got):
                want = O.query(g, p, 20, 1.0, O.FULL)
                for k in FULL_KEYS:
                    assert r[k] == want[k], (fused, p, k, r[k], want[k])
        small.set("chain_queries", 64)
        small.set("chain_steps", 8)
        with small.load_graph(g) as dg:
            _say("forms fused", fused, "chains", len(pats))
            got = dg.support_batch(pats, [20] * len(pats), [1.0] * len(pats), fx.MODE_FULL)
            for p, r in zip(pats, got):
                want = O.query(g, p, 20, 1.0, O.FULL)
                for k in FULL_KEYS:
                    assert r[k] == want[k], (fused, p, k, r[k], want[k])
        assert small.stats()["chains"] > 0
        small.close()
        big.close()
