"""The allocation-free entry point (fx_support_noalloc) against fx_support.

Two calls in a row, the second with a smaller input, in every mode; the
results must equal fx_support's exactly (every field is an integer), and the
library's count of device and pinned-host allocation calls must not move
during the allocation-free calls."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2404_01585_amd import flexis as fx
from paper_2404_01585_amd.synth import Pattern, sample_patterns, workload_graph

pytestmark = pytest.mark.gpu

KEYS = ("tau", "support", "frequent", "embedding_count", "count_saturated", "digest", "sel_digest", "exit", "status")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_noalloc_equals_support(torch_cuda):
    g = workload_graph("er1k")
    big = sample_patterns(g, 6, seed=71, kmin=5, kmax=7)
    small = sample_patterns(g, 6, seed=72, kmin=2, kmax=3)
    with fx.Context(device=0) as ctx, ctx.load_graph(g) as dg:
        for mode in (fx.MODE_FULL, fx.MODE_VERDICT, fx.MODE_MNI):
            for first, second in zip(big, small):
                want = [dg.support(p, 20, 0.5, mode) for p in (first, second)]
                a0 = fx.alloc_calls()
                got = [dg.support_noalloc(p, 20, 0.5, mode) for p in (first, second)]
                assert fx.alloc_calls() == a0, "an allocation-free call allocated"
                _say("noalloc mode", mode, "n", first.n, "then", second.n)
                for w, r in zip(want, got):
                    for k in KEYS:
                        assert r[k] == w[k], (mode, k, r[k], w[k])
        # and against the oracle directly, two calls in a row
        for p in (big[0], small[0]):
            want = O.query(g, p, 20, 1.0, O.FULL)
            r = dg.support_noalloc(p, 20, 1.0, fx.MODE_FULL)
            for k in ("tau", "support", "frequent", "embedding_count", "digest", "sel_digest"):
                assert r[k] == want[k], (k, r[k], want[k])


def test_noalloc_larger_graph_and_limit(torch_cuda):
    # the 100K-vertex graph: a stack with a used-vertex bitmap of 12.5 KB;
    # then a pattern whose stack cannot fit the scratch array is refused
    g = workload_graph("cl100k")
    pats = sample_patterns(g, 4, seed=73, kmin=3, kmax=5)
    with fx.Context(device=0, no_digest=True) as ctx, ctx.load_graph(g) as dg:
        for p in pats:
            w = dg.support(p, 200, 1.0, fx.MODE_VERDICT)
            a0 = fx.alloc_calls()
            r = dg.support_noalloc(p, 200, 1.0, fx.MODE_VERDICT)
            assert fx.alloc_calls() == a0
            _say("noalloc cl100k n", p.n)
            for k in KEYS:
                assert r[k] == w[k], (k, r[k], w[k])
        # a 16-vertex path: 15 levels of 2^14 rows, about 12 MB: fits
        path = Pattern([0] * 16, [(i, i + 1) for i in range(15)], [0] * 15)
        r = dg.support_noalloc(path, 1000, 1.0, fx.MODE_VERDICT)
        w = dg.support(path, 1000, 1.0, fx.MODE_VERDICT)
        assert (r["frequent"], r["support"]) == (w["frequent"], w["support"])
    # MNI mode on a graph large enough that 17 bitmaps of |V|/8 bytes do not fit
    from paper_2404_01585_amd.synth import Graph
    nv = 1 << 25
    chain_col = np.array([1, 0], dtype=np.int32)
    gl = Graph(row_ptr=np.concatenate([[0, 1, 2], np.full(nv - 2, 2)]).astype(np.int64), col=chain_col,
               vlabel=np.zeros(nv, dtype=np.int32), elabel=np.zeros(2, dtype=np.int32))
    with fx.Context(device=0) as ctx, ctx.load_graph(gl) as dg:
        p16 = Pattern([0] * 16, [(i, i + 1) for i in range(15)], [0] * 15)
        with pytest.raises(fx.FxError) as e:
            dg.support_noalloc(p16, 1, 1.0, fx.MODE_MNI)
        assert e.value.status == fx.FX_ELIMIT
        # and the entry point still works afterwards on the same device
        r = dg.support_noalloc(Pattern([0, 0], [(0, 1)], [0]), 1, 1.0, fx.MODE_FULL)
        assert r["support"] == 1 and r["embedding_count"] == 2
