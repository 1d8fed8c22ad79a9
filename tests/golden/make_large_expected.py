"""Writes the oracle's results for sampled patterns on the full-size graphs.

Calls only the CPU oracle (``oracle/``) and the seeded input generators; no
value here comes from the device path.  Each pattern is answered in a worker
process under a time limit; patterns the oracle does not finish in time are
left out of the file (the selection is recorded, not re-derived).

    python tests/golden/make_large_expected.py [--workers 8] [--limit 120] [--set large|cl100k]

Output: tests/golden/large_expected.json (the 1M-vertex Chung-Lu and 4M-vertex
R-MAT sets) or tests/golden/cl100k_expected.json (the 100K-vertex Chung-Lu set).
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

COUNT_CAP = 10 ** 7

_G = {}


def _graph(name):
    from paper_2404_01585_amd.synth import workload_graph
    from oracle import oracle as O

    if name not in _G:
        _G[name] = O.OracleGraph.of(workload_graph(name))
    return _G[name]


def _answer(args):
    name, pat, sigma, lam = args
    from oracle import oracle as O
    from paper_2404_01585_amd.synth import Pattern

    g = _graph(name)
    p = Pattern(**pat)
    t = time.time()
    full = O.query(g, p, sigma, lam, O.FULL, count_cap=COUNT_CAP)
    ver = O.query(g, p, sigma, lam, O.VERDICT)
    return dict(graph=name, pattern=pat, sigma=sigma, lam=lam,
                full=dict(tau=full["tau"], support=full["support"], frequent=full["frequent"],
                          embedding_count=full["embedding_count"], count_saturated=full["count_saturated"],
                          digest=list(full["digest"])),
                verdict=dict(tau=ver["tau"], support=ver["support"], frequent=ver["frequent"]),
                oracle_s=round(time.time() - t, 3))


def _cases_cl100k():
    import numpy as np

    from paper_2404_01585_amd.synth import sample_patterns, workload_graph

    out = []
    rng = np.random.default_rng(2027)
    # 100K-vertex Chung-Lu with 3 edge labels: 200 sampled patterns of each size
    # 2, 3 and 4 (the sizes of mining levels 1-3), sigma 200, lambda 0.3 or 1.0
    g = workload_graph("cl100k")
    for k in (2, 3, 4):
        for p in sample_patterns(g, 200, seed=60 + k, kmin=k, kmax=k):
            out.append(("cl100k", dict(vlabel=p.vlabel, edges=[list(e) for e in p.edges], elabel=p.elabel), 200,
                        float(rng.choice([0.3, 1.0]))))
    return out


def _cases():
    import numpy as np

    from paper_2404_01585_amd.synth import sample_patterns, workload_graph

    out = []
    rng = np.random.default_rng(2026)
    # 1M-vertex Chung-Lu: the sampled-pattern batch (3-7 vertices), sigma 200
    g = workload_graph("cl1m")
    for p in sample_patterns(g, 2000, seed=33, kmin=3, kmax=7)[:160]:
        out.append(("cl1m", dict(vlabel=p.vlabel, edges=[list(e) for e in p.edges], elabel=p.elabel), 200,
                    float(rng.choice([0.1, 0.5, 1.0]))))
    # 4M-vertex R-MAT: labeled edges and sampled 3-4-vertex patterns, sigma 2000
    g = workload_graph("rmat22")
    for p in sample_patterns(g, 120, seed=55, kmin=2, kmax=4):
        out.append(("rmat22", dict(vlabel=p.vlabel, edges=[list(e) for e in p.edges], elabel=p.elabel), 2000,
                    float(rng.choice([0.1, 0.5, 1.0]))))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--limit", type=float, default=120.0, help="seconds per pattern")
    ap.add_argument("--set", default="large", choices=["large", "cl100k"])
    args = ap.parse_args()
    cases = _cases() if args.set == "large" else _cases_cl100k()
    for name in sorted({c[0] for c in cases}):
        _graph(name)  # built once here; the forked workers share it
    results, skipped = [], []
    ctx = mp.get_context("fork")
    for start in range(0, len(cases), args.workers):
        chunk = cases[start:start + args.workers]
        with ctx.Pool(len(chunk), maxtasksperchild=1) as pool:
            futs = [pool.apply_async(_answer, (c,)) for c in chunk]
            t0 = time.time()
            for c, f in zip(chunk, futs):
                try:
                    results.append(f.get(timeout=max(1.0, args.limit - (time.time() - t0))))
                except mp.TimeoutError:
                    skipped.append(dict(graph=c[0], pattern=c[1]))
            pool.terminate()
        print(f"{start + len(chunk)}/{len(cases)} done, {len(skipped)} skipped", flush=True)
    name = "large_expected.json" if args.set == "large" else "cl100k_expected.json"
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(dict(count_cap=COUNT_CAP, results=results, skipped=skipped), f)
    print(len(results), "stored")


if __name__ == "__main__":
    main()
