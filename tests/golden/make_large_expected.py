"""Writes the oracle's results for sampled patterns on the full-size graphs.

Calls only the CPU oracle (``oracle/``) and the seeded input generators; no
value here comes from the device path.  Each pattern is answered in a worker
process of its own under a time limit (the paper stops a mining run after 30
minutes, Section 4.1; the same limit per pattern is the default here);
patterns the oracle does not finish in time are stored under ``unfinished``
with their sigma, lambda and the limit, so the selection is recorded, not
re-derived.

    python tests/golden/make_large_expected.py --set large  [--workers 6] [--limit 1800]
    python tests/golden/make_large_expected.py --set cl100k [--workers 6] [--limit 600]
    python tests/golden/make_large_expected.py --set digest [--workers 6] [--limit 900]

``large``  -> large_expected.json: the 1M-vertex Chung-Lu and 4M-vertex R-MAT
              sets; FULL (count capped at 10^7) with the selected set's digest,
              and VERDICT.
``cl100k`` -> cl100k_expected.json: the 100K-vertex Chung-Lu set.
``digest`` -> large_digest_expected.json: the cases of large_expected.json
              whose count saturated at 10^7, counted again with the cap at
              10^9, so that the embedding-set digest can be compared where
              the count stays below it.
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
DIGEST_CAP = 10 ** 9

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
                          digest=list(full["digest"]), sel_digest=list(full["sel_digest"])),
                verdict=dict(tau=ver["tau"], support=ver["support"], frequent=ver["frequent"]),
                oracle_s=round(time.time() - t, 3))


def _answer_count(args):
    name, pat, sigma, lam = args
    from oracle import oracle as O
    from paper_2404_01585_amd.synth import Pattern

    g = _graph(name)
    t = time.time()
    c, sat, dg = O.count(g, Pattern(**pat), DIGEST_CAP)
    return dict(graph=name, pattern=pat, sigma=sigma, lam=lam,
                full=dict(embedding_count=c, count_saturated=int(sat), digest=list(dg) if not sat else [0, 0]),
                oracle_s=round(time.time() - t, 3))


def _pat(p):
    return dict(vlabel=[int(x) for x in p.vlabel], edges=[[int(a), int(b)] for a, b in p.edges],
                elabel=[int(x) for x in p.elabel])


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
            out.append(("cl100k", _pat(p), 200, float(rng.choice([0.3, 1.0]))))
    return out


def _cases():
    import numpy as np

    from paper_2404_01585_amd.synth import sample_patterns, workload_graph

    out = []
    rng = np.random.default_rng(2026)
    # 1M-vertex Chung-Lu: the sampled-pattern batch (3-7 vertices), sigma 200
    g = workload_graph("cl1m")
    for p in sample_patterns(g, 2000, seed=33, kmin=3, kmax=7)[:160]:
        out.append(("cl1m", _pat(p), 200, float(rng.choice([0.1, 0.5, 1.0]))))
    # 4M-vertex R-MAT: labeled edges and sampled 3-4-vertex patterns, sigma 2000
    g = workload_graph("rmat22")
    for p in sample_patterns(g, 120, seed=55, kmin=2, kmax=4):
        out.append(("rmat22", _pat(p), 2000, float(rng.choice([0.1, 0.5, 1.0]))))
    return out


def _cases_digest():
    with open(os.path.join(HERE, "large_expected.json")) as f:
        done = json.load(f)
    return [(r["graph"], r["pattern"], r["sigma"], r["lam"]) for r in done["results"]
            if r["full"]["count_saturated"]]


def _worker(fn, case, conn):
    try:
        conn.send(("ok", fn(case)))
    except BaseException as e:  # reported, never swallowed
        conn.send(("error", repr(e)))
    conn.close()


def run_all(cases, fn, workers, limit):
    """Answers every case in its own forked process, at most `workers` at
    once; a case still running after `limit` seconds is killed and listed
    as unfinished.  Results keep the order of `cases`."""
    ctx = mp.get_context("fork")
    results = [None] * len(cases)
    unfinished = []
    running = {}  # index -> (process, conn, start)
    nxt = 0
    finished = 0
    while nxt < len(cases) or running:
        while nxt < len(cases) and len(running) < workers:
            a, b = ctx.Pipe(duplex=False)
            pr = ctx.Process(target=_worker, args=(fn, cases[nxt], b))
            pr.start()
            b.close()
            running[nxt] = (pr, a, time.time())
            nxt += 1
        time.sleep(0.05)
        for i in list(running):
            pr, conn, t0 = running[i]
            if conn.poll():
                kind, val = conn.recv()
                pr.join()
                if kind != "ok":
                    raise RuntimeError(f"case {i} failed in the oracle: {val}")
                results[i] = val
            elif time.time() - t0 > limit:
                pr.kill()
                pr.join()
                c = cases[i]
                unfinished.append(dict(graph=c[0], pattern=c[1], sigma=c[2], lam=c[3], limit_s=limit))
            elif not pr.is_alive():
                raise RuntimeError(f"case {i}: worker ended without a result (exit code {pr.exitcode})")
            else:
                continue
            conn.close()
            del running[i]
            finished += 1
            print(f"{finished}/{len(cases)} done, {len(unfinished)} unfinished "
                  f"(case {i}: {'%.1f s' % (time.time() - t0)})", flush=True)
    return [r for r in results if r is not None], unfinished


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--limit", type=float, default=1800.0, help="seconds per pattern")
    ap.add_argument("--set", default="large", choices=["large", "cl100k", "digest"])
    args = ap.parse_args()
    if args.set == "large":
        cases, fn, name, cap = _cases(), _answer, "large_expected.json", COUNT_CAP
    elif args.set == "cl100k":
        cases, fn, name, cap = _cases_cl100k(), _answer, "cl100k_expected.json", COUNT_CAP
    else:
        cases, fn, name, cap = _cases_digest(), _answer_count, "large_digest_expected.json", DIGEST_CAP
    for g in sorted({c[0] for c in cases}):
        _graph(g)  # built once here; the forked workers share it
    t0 = time.time()
    results, unfinished = run_all(cases, fn, args.workers, args.limit)
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(dict(count_cap=cap, limit_s=args.limit, results=results, unfinished=unfinished), f)
    print(len(results), "stored,", len(unfinished), "unfinished,", round(time.time() - t0), "s")


if __name__ == "__main__":
    main()
