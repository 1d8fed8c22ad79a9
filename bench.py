#!/usr/bin/env python3
"""Support-counting throughput on one MI355X.

A step is one pass of the whole hot path over one batch of candidate
patterns: for every pattern, enumerate its embeddings, take the greedy
maximal independent set, compare it with tau, and count the embeddings
(FULL mode), all through the C ABI of libflexis.so.

Default workload ("rmat22-sweep"): R-MAT graph of scale 22 (4,194,304
vertices, 40M undirected edges, a,b,c = 0.57,0.19,0.19), 50 vertex labels
Zipf(1.1), 4 edge labels uniform, int64 row offsets; sigma = 2000 with the
lambda sweep {0.1, 0.5, 1.0}.  For each lambda the batch is every candidate of
the first two levels of the mining loop (Algorithm 1): all labeled edges and
every one-edge extension of the frequent ones (the loop itself runs untimed
before the timed region).  Step k evaluates the batch of lambda number
k mod 3, so the timed steps cycle through the sweep.  Inputs are synthetic and
seeded; the graph is resident in HBM before the timed region.

Prints one JSON line: patterns/s over the timed steps, the roofline of every
expansion and greedy kernel from a one-lane pass after the timed region (HIP
events on the lane's stream around every launch; reference algorithmic bytes
from a second, counting pass with the same launches), and the CPU oracle's
rate on a bounded sample of the same batches.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Launch shape per workload (fx_ctx_set tunables), chosen with fx_autotune on
# the MI355X; --autotune re-tunes instead, the shape flags override.
SHAPE_RMAT22 = dict(slice_rows=1 << 16, step_candidates=1 << 26, items_per_thread=4, last_span_init=4096, lanes=2,
                    max_active=4096)
SHAPE_CL100K = dict(slice_rows=1 << 17, step_candidates=1 << 25, items_per_thread=4, last_span_init=4096, lanes=2,
                    max_active=4096)

WORKLOADS = {
    "rmat22-sweep": dict(graph="rmat22", sigma=2000, lams=[0.1, 0.5, 1.0], levels=2, shape=SHAPE_RMAT22,
                         desc="R-MAT scale 22 (4,194,304 vertices, 40M edges, a,b,c = 0.57,0.19,0.19), 50 Zipf(1.1) "
                              "vertex labels, 4 edge labels, int64 offsets; sigma=2000, lambda sweep {0.1, 0.5, "
                              "1.0}; per lambda every candidate of mining levels 1-2; step k runs the batch of "
                              "lambda k mod 3"),
    "rmat22-l2": dict(graph="rmat22", sigma=2000, lams=[1.0], levels=2, shape=SHAPE_RMAT22,
                      desc="R-MAT scale 22 (4,194,304 vertices, 40M edges, a,b,c = 0.57,0.19,0.19), 50 Zipf(1.1) "
                           "vertex labels, 4 edge labels, int64 offsets; all candidates of mining levels 1-2 at "
                           "sigma=2000, lambda=1.0"),
    "cl100k-l2": dict(graph="cl100k", sigma=200, lams=[1.0], levels=2, shape=SHAPE_CL100K,
                      desc="Chung-Lu 100K vertices / 500K edges (gamma 2.1), 20 Zipf(1.2) vertex labels, "
                           "3 edge labels; all candidates of mining levels 1-2 at sigma=200, lambda=1.0"),
    "cl100k-l2-sweep": dict(graph="cl100k", sigma=200, lams=[0.3, 1.0], levels=2, shape=SHAPE_CL100K,
                            desc="Chung-Lu 100K vertices / 500K edges (gamma 2.1), 20 Zipf(1.2) vertex labels, "
                                 "3 edge labels; sigma=200, lambda in {0.3, 1.0}; per lambda every candidate of "
                                 "mining levels 1-2"),
    "cl100k-l3": dict(graph="cl100k", sigma=200, lams=[1.0], levels=3, shape=SHAPE_CL100K,
                      desc="Chung-Lu 100K vertices / 500K edges (gamma 2.1), 20 Zipf(1.2) vertex labels, "
                           "3 edge labels; all candidates of mining levels 1-3 at sigma=200, lambda=1.0"),
    "cl1m-s2000": dict(graph="cl1m", sigma=200, lams=[1.0], sample=dict(count=2000, seed=33, kmin=3, kmax=7),
                       desc="Chung-Lu 1M vertices / 8M edges (gamma 2.3), 30 Zipf(1.0) vertex labels, 1 edge "
                            "label; 2,000 patterns of 3-7 vertices (trees, cycles, trees plus a chord) sampled "
                            "as connected subgraphs of the graph, sigma=200, lambda=1.0"),
    "cl100k-v4": dict(graph="cl100k", sigma=200, lams=[1.0], vertices=4, shape=SHAPE_CL100K,
                      desc="Chung-Lu 100K vertices / 500K edges (gamma 2.1), 20 Zipf(1.2) vertex labels, "
                           "3 edge labels; all candidates of the merge generator (levels by vertex count) up to "
                           "4 vertices at sigma=200, lambda=1.0"),
    "er1k-l4": dict(graph="er1k", sigma=20, lams=[1.0], levels=4,
                    desc="Erdos-Renyi 1K vertices / 4K edges, 5 uniform vertex labels, 1 edge label; all "
                         "candidates of mining levels 1-4 at sigma=20, lambda=1.0"),
}
DEFAULT_WORKLOAD = "rmat22-sweep"
GRAPH_DESC = {"cl100k": "Chung-Lu 100K vertices / 500K edges (gamma 2.1), 20 Zipf(1.2) vertex labels, 3 edge labels",
              "rmat22": "R-MAT scale 22 (4,194,304 vertices, 40M edges), 50 Zipf(1.1) vertex labels, 4 edge labels",
              "cl1m": "Chung-Lu 1M vertices / 8M edges (gamma 2.3), 30 Zipf(1.0) vertex labels, 1 edge label"}
SHAPE_KEYS = ("slice_rows", "step_candidates", "items_per_thread", "last_span_init", "lanes", "max_active")
ENGINE_KEYS = ("chain_queries", "chain_steps", "fused", "fused_below")  # engine choices (library defaults unless given)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_candidates(dg, g, spec, lam, types=None):
    """Candidate batch for one lambda: patterns sampled from the graph, or
    every candidate of the first `levels` mining levels (the level-wise loop
    itself runs here, untimed, with verdicts from the device path)."""
    from paper_2404_01585_amd import flexis as fx
    from paper_2404_01585_amd import mining
    from paper_2404_01585_amd.synth import sample_patterns

    if "sample" in spec:
        sm = spec["sample"]
        cands = sample_patterns(g, sm["count"], seed=sm["seed"], kmin=sm["kmin"], kmax=sm["kmax"])
        return cands, [len(cands)]

    def evaluate(ps, sigma, l):
        return dg.support_batch(ps, [sigma] * len(ps), [l] * len(ps), fx.MODE_VERDICT)

    if "vertices" in spec:  # Algorithm 1 with the merge generator (Algorithms 2-4)
        from paper_2404_01585_amd import generate

        res = generate.mine_by_vertices(g, spec["sigma"], lam, spec["vertices"], evaluate, fx.tau)
    else:
        # the last level's candidates are the batch itself: generated, not evaluated here
        res = mining.mine(g, spec["sigma"], lam, spec["levels"], evaluate, tau_fn=fx.tau, types=types,
                          evaluate_last=False)
    cands = [p for lvl in res["levels"] for p in lvl]
    return cands, [len(l) for l in res["levels"]]


def traffic_from_profile(kernel_src: str, workload: str):
    """HBM traffic per probe launch from the committed PMC summary of this
    workload, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_probe_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sha256") != hashlib.sha256(open(kernel_src, "rb").read()).hexdigest():
        return None
    return t.get("bytes_per_launch")


_CPU = {}


def _cpu_start(barrier):
    _CPU["barrier"] = barrier


def _cpu_load(path):
    """Reads the graph and the batch the parent wrote, then waits for every
    other worker (so each worker loads exactly once, before any timed task)."""
    from oracle import oracle as O

    z = np.load(path)
    _CPU.update(g=O.OracleGraph(z["row_ptr"], z["col"], z["vlabel"], z["elabel"]),
                pats=[O.OraclePattern(p["vlabel"], p["edges"], p["elabel"]) for p in json.loads(str(z["patterns"]))],
                sigma=[int(x) for x in z["sigma"]], lam=[float(x) for x in z["lam"]])
    _CPU["barrier"].wait(timeout=900)
    return os.getpid()


def _cpu_task(i):
    """One FULL-mode oracle query; returns its own start and end time."""
    from oracle import oracle as O

    t0 = time.time()
    O.query(_CPU["g"], _CPU["pats"][i], _CPU["sigma"][i], _CPU["lam"][i], O.FULL)
    return i, t0, time.time()


def start_cpu_pool(threads: int):
    """Worker processes of the CPU baseline, started before this process
    touches the GPU (they never do)."""
    import multiprocessing as mp

    ctx = mp.get_context("spawn")
    return ctx.Pool(threads, initializer=_cpu_start, initargs=(ctx.Barrier(threads),))


def cpu_baseline(pool, threads: int, g, cands, sigmas, lams, seconds: float):
    """The oracle (untuned) on the host cores: FULL-mode queries (support,
    count and digest) over the batch in order, one per worker process, for
    about `seconds` after every worker has read the graph.  value = queries
    finished by the deadline over the wall time since the first query
    started; single_core_value = those queries over the sum of their own
    durations (each ran on one core)."""
    import multiprocessing as mp
    import tempfile

    fd, path = tempfile.mkstemp(suffix=".npz", prefix="fx_cpu_")
    os.close(fd)
    try:
        pats = [dict(vlabel=list(map(int, p.vlabel)), edges=[list(map(int, e)) for e in p.edges],
                     elabel=list(map(int, p.elabel))) for p in cands]
        with open(path, "wb") as f:
            np.savez(f, row_ptr=g.row_ptr, col=g.col, vlabel=g.vlabel, elabel=g.elabel,
                     patterns=np.array(json.dumps(pats)), sigma=np.asarray(sigmas, dtype=np.int64),
                     lam=np.asarray(lams, dtype=np.float64))
        try:
            pids = pool.map(_cpu_load, [path] * threads, chunksize=1)
            it = pool.imap_unordered(_cpu_task, range(len(cands)))
            first, deadline = None, None
            busy, done = 0.0, 0
            while True:
                try:
                    timeout = None if deadline is None else deadline - time.time()
                    if timeout is not None and timeout <= 0:
                        break
                    _, t0, t1 = it.next(timeout=timeout)
                except (StopIteration, mp.TimeoutError):
                    break
                if first is None or t0 < first:
                    first = t0
                    deadline = first + seconds
                if t1 <= deadline:
                    done += 1
                    busy += t1 - t0
            wall = (min(time.time(), deadline) - first) if first is not None else 0.0
        finally:
            pool.terminate()
            pool.join()
    finally:
        os.unlink(path)
    return dict(value=done / wall if wall > 0 else 0.0, unit="patterns/s", cores=len(set(pids)), kind="oracle",
                single_core_value=round(done / busy, 3) if busy > 0 else None,
                sample=f"{done} of {len(cands)} candidates of the timed batches (taken in batch order) finished in "
                       f"{wall:.1f} s wall on {len(set(pids))} processes, FULL mode; the oracle also hashes every "
                       f"embedding for the digest, while the timed GPU steps count without hashing "
                       f"(leaf-ended patterns in closed form)")


def serving_queries(g, count: int, seed: int, kmax: int = 8):
    """Support queries of the serving workload: patterns of 3-kmax vertices
    sampled from the graph, sigma log-uniform in [50, 5000], lambda uniform in
    {0.1, 0.5, 1.0}."""
    import numpy as np

    from paper_2404_01585_amd.synth import sample_patterns

    rng = np.random.default_rng(seed)
    pats = sample_patterns(g, count, seed=seed, kmin=3, kmax=kmax)
    sig = np.floor(np.exp(rng.uniform(np.log(50), np.log(5001), size=count))).astype(np.int64)
    lam = rng.choice([0.1, 0.5, 1.0], size=count)
    return pats, [int(x) for x in sig], [float(x) for x in lam]


def _lat_summary(lat_ms, n, wall):
    import numpy as np
    a = np.asarray(lat_ms)
    return dict(n=n, p50_ms=round(float(np.percentile(a, 50)), 3), p99_ms=round(float(np.percentile(a, 99)), 3),
                throughput_qps=round(n / wall, 1))


def run_served(srv, queries, rate: float, mode: int, seed: int):
    """Open-loop Poisson arrivals into the server; latency = submit -> result
    (measured by the library)."""
    import numpy as np
    pats, sig, lam = queries
    n = len(pats)
    arr = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=n))
    t0 = time.perf_counter()
    tickets = []
    for i in range(n):
        wait = t0 + arr[i] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        tickets.append(srv.submit(pats[i], sig[i], lam[i], mode))
        if (i + 1) % 2000 == 0 and i + 1 < n:
            log(f"[serve] {i + 1}/{n} submitted at {rate} q/s")
    log(f"[serve] {n} submitted at {rate} q/s")
    res = []
    last = time.perf_counter()
    for k, t in enumerate(tickets):
        while True:  # a long query: report the server's device steps meanwhile
            r = srv.poll(t)
            if r is not None:
                break
            time.sleep(0.0005)
            if time.perf_counter() - last > 15.0:
                last = time.perf_counter()
                log(f"[serve] {k}/{n} answered, {srv.stats()['steps']} server device steps so far")
        res.append(r)
        if (k + 1) % 1000 == 0:
            log(f"[serve] {k + 1}/{n} answered")
    wall = time.perf_counter() - t0
    return _lat_summary([r["device_ms"] for r in res], n, wall), res


def run_fifo(dg, queries, rate: float, mode: int, seed: int):
    """The same arrivals served one query per call, first come first served;
    latency = completion - arrival."""
    import numpy as np
    pats, sig, lam = queries
    n = len(pats)
    arr = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=n))
    t0 = time.perf_counter()
    lat, res = [], []
    for i in range(n):
        wait = t0 + arr[i] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        res.append(dg.support(pats[i], sig[i], lam[i], mode))
        lat.append((time.perf_counter() - (t0 + arr[i])) * 1e3)
        if (i + 1) % 500 == 0:
            log(f"[fifo] {i + 1}/{n} answered")
    wall = time.perf_counter() - t0
    return _lat_summary(lat, n, wall), res


def serve_sweep(args):
    """Serving workload: the cl100k graph resident, Poisson streams of support
    queries at several rates; continuous batching vs one query per call, in
    VERDICT and FULL modes.  Prints one JSON line."""
    import torch

    from paper_2404_01585_amd import flexis as fx
    from paper_2404_01585_amd.synth import workload_graph

    g = workload_graph(args.serve_graph)
    torch.cuda.set_device(0)
    ctx = fx.Context(device=0, no_digest=True, count_cap=args.serve_count_cap)
    dg = ctx.load_graph(g)
    queries = serving_queries(g, args.serve_queries, seed=4, kmax=args.serve_kmax)
    log(f"[serve] {len(queries[0])} queries sampled from {args.serve_graph}")
    out = []
    plan = (("verdict", fx.MODE_VERDICT, args.serve_rates, queries),
            ("full", fx.MODE_FULL, args.serve_full_rates, tuple(x[:args.serve_full_queries] for x in queries)))
    for mode_name, mode, rate_list, qset in plan:
        rates = [float(r) for r in rate_list.split(",") if r]
        with fx.Server(dg, no_digest=True, step_candidates=args.serve_step) as srv:
            run_served(srv, tuple(x[:100] for x in qset), 1000.0, mode, seed=99)  # warm the server
            for rate in rates:
                queries = qset
                served, res_s = run_served(srv, queries, rate, mode, seed=int(rate))
                row = dict(mode=mode_name, rate_qps=rate, served=served)
                if not args.no_fifo:
                    fifo, res_f = run_fifo(dg, queries, rate, mode, seed=int(rate))
                    row["fifo_one_per_call"] = fifo
                    row["same_results"] = all(a["frequent"] == b["frequent"] and a["support"] == b["support"]
                                              for a, b in zip(res_s, res_f))
                log(f"[serve] {row}")
                out.append(row)
    line = {"metric": "p50/p99 support-query latency and throughput at 1 GPU (served, continuous batching)",
            "unit": "ms", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": f"{args.serve_graph}-serve: {GRAPH_DESC[args.serve_graph]} resident; Poisson "
                                   f"arrivals; patterns of 3-{args.serve_kmax} vertices sampled from the graph; sigma log-uniform "
                                   "[50, 5000]; lambda in {0.1, 0.5, 1.0}", "queries_per_rate_verdict": args.serve_queries,
                       "queries_per_rate_full": args.serve_full_queries, "count_cap_full": args.serve_count_cap,
                       "step_candidates": args.serve_step},
            "rates": out}
    print(json.dumps(line), flush=True)
    dg.close()
    ctx.close()


def apply_shape(ctx, shape: dict):
    for k in SHAPE_KEYS:
        if shape.get(k) is not None:
            ctx.set(k, int(shape[k]))


def marker():
    """A tiny torch fill kernel: in a kernel trace it marks where the one-lane
    roofline pass starts and ends (the library launches no torch kernels)."""
    import torch

    torch.cuda.synchronize()
    torch.empty(1, device="cuda").fill_(1.0)
    torch.cuda.synchronize()


KERNELS = (("probe", "k_probe"), ("scatter", "k_scatter"), ("greedy", "k_greedy"))
FUSED_KERNELS = (("probe", "k_expand"), ("greedy", "k_greedy"))  # the single-pass expansion: probe and write


def roofline_pass(ctx, dg, batches, mode, repeats: int, count_ref: bool, traffic):
    """Per-kernel roofline of the expansion and greedy kernels: the batches run
    once more with one lane (no other stream's kernels overlap them) and HIP
    events around every launch; then, when count_ref, again with the same
    launches and the reference algorithmic bytes counted on the device (extra
    loads, so never in the timed pass)."""
    lanes0, chain0, below0 = ctx.get("lanes"), ctx.get("chain_queries"), ctx.get("fused_below")
    ctx.set("lanes", 1)
    ctx.set("chain_queries", 0)  # both passes host-scheduled, so their launches are the same
    ctx.set("fused_below", 0)    # and every step of one form
    marker()
    ctx.set("kernel_timing", 1)
    ctx.stats(reset=True)
    for r in range(repeats):
        for lam, b in batches:
            dg.support_batch_array(b, b.sigma, lam, mode)
        log(f"[bench] roofline timing pass {r + 1}/{repeats} done")
    st = ctx.stats(reset=True)
    ctx.set("kernel_timing", 0)
    marker()
    ref = None
    if count_ref:
        ctx.set("ref_bytes", 1)
        for r in range(repeats):
            for lam, b in batches:
                dg.support_batch_array(b, b.sigma, lam, mode)
        ref = ctx.stats(reset=True)
        ctx.set("ref_bytes", 0)
        log("[bench] roofline counting pass done")
    ctx.set("lanes", lanes0)
    ctx.set("chain_queries", chain0)
    ctx.set("fused_below", below0)
    per = {}
    fused = bool(ctx.get("fused"))
    for key, name in (FUSED_KERNELS if fused else KERNELS):
        n = st[f"{key}_launches"]
        if not n or st[f"{key}_ms"] <= 0:
            continue
        avg_s = st[f"{key}_ms"] / n * 1e-3
        d = dict(kernel=name, launches=n, avg_launch_us=round(avg_s * 1e6, 3))
        if ref is not None and ref[f"{key}_launches"] == n:
            rb = ref[f"{key}_ref_bytes"] / n
            if fused and key == "probe":  # the fused kernel also writes the rows
                rb += ref["scatter_ref_bytes"] / n
            d.update(ref_bytes_per_launch=round(rb, 1), achieved=round(rb / avg_s / 1e9, 3),
                     frac=round(rb / avg_s / 1e9 / HBM_PEAK_GBS, 6))
            if key == "probe":  # the same model for plain (not label-sorted) rows
                rr = ref["probe_ref_row_bytes"] / n
                d.update(plain_row_model_bytes_per_launch=round(rr, 1),
                         plain_row_model_frac=round(rr / avg_s / 1e9 / HBM_PEAK_GBS, 6))
        elif ref is not None:
            d.update(ref_launches_differ=ref[f"{key}_launches"])
        if key in ("probe", "scatter"):
            tb = st[f"{key}_alg_bytes"] / n
            if fused and key == "probe":
                tb += st["scatter_alg_bytes"] / n
            d.update(touched_bytes_per_launch=round(tb, 1), touched_frac=round(tb / avg_s / 1e9 / HBM_PEAK_GBS, 6))
        per[key] = d
    if "probe" not in per:
        return None
    p = per["probe"]
    return dict(bound="hbm", achieved=p.get("achieved"), peak=HBM_PEAK_GBS, unit="GB/s", frac=p.get("frac"),
                traffic=traffic, kernel=p["kernel"], avg_launch_us=p["avg_launch_us"],
                alg_bytes_per_launch=p.get("ref_bytes_per_launch"), launches=p["launches"], per_kernel=per,
                timing="one-lane pass after the timed region (the same batches, host-scheduled steps, HIP events "
                       "around every launch on the lane's stream); algorithmic bytes = reference bytes counted on "
                       "the device in a second pass with the same launches")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="full", choices=["full", "verdict"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--count-cap", type=int, default=0, help="embedding count cap (0: 2^62)")
    ap.add_argument("--no-run-index", action="store_true",
                    help="no label-run index: candidate runs and edge tests by binary search in the rows")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="run the autotuner (untimed) instead of the fixed shape")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (with --autotune)")
    for k in SHAPE_KEYS:
        ap.add_argument("--" + k.replace("_", "-"), type=int, default=None,
                        help=f"launch shape: {k} (default: the workload's tuned value)")
    for k in ENGINE_KEYS:
        ap.add_argument("--" + k.replace("_", "-"), type=int, default=None,
                        help=f"engine tunable {k} (default: the library's)")
    ap.add_argument("--digest", action="store_true",
                    help="also hash every embedding (FULL-mode digest); counts are exact either way")
    ap.add_argument("--plain-seconds", type=float, default=5.0,
                    help="time the one-pattern-per-call form on a prefix of the batches for this long")
    ap.add_argument("--roofline-repeats", type=int, default=1, help="passes over the batches in the roofline pass")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--profile-pass", action="store_true",
                    help="for a kernel trace: graph, candidates and the one-lane timing pass only (no timed "
                         "steps, no counting pass, no plain form, serving probe or CPU baseline)")
    ap.add_argument("--serve", action="store_true", help="serving sweep (Poisson arrivals) instead of the batch")
    ap.add_argument("--serve-graph", default="cl100k", choices=sorted(GRAPH_DESC))
    ap.add_argument("--serve-rates", default="100,300,1000,3000,5000")
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--serve-full-rates", default="100,1000")
    ap.add_argument("--serve-full-queries", type=int, default=300)
    ap.add_argument("--serve-count-cap", type=int, default=10 ** 9)
    ap.add_argument("--serve-step", type=int, default=1 << 22, help="candidates per device step of the server")
    ap.add_argument("--no-fifo", action="store_true")
    ap.add_argument("--serve-kmax", type=int, default=8, help="largest pattern size of the serving queries")
    ap.add_argument("--serve-probe-rate", type=float, default=1000.0,
                    help="rate of the short serving probe in the default run (0: skip)")
    ap.add_argument("--serve-probe-queries", type=int, default=1000)
    ap.add_argument("--serve-probe-graph", default="cl100k", choices=sorted(GRAPH_DESC),
                    help="graph of the serving probe (the serving configuration's own graph by default)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="calibration only: copy a buffer of this many bytes 5 times with torch and exit "
                         "(a plain copy kernel of known size for the PMC traffic factors)")
    ap.add_argument("--gather-count", type=int, default=0,
                    help="calibration only: gather this many random 8-byte words from a 4 GiB table 5 times "
                         "with torch and exit (random reads of known count for the PMC traffic factors)")
    args = ap.parse_args()

    if args.serve:
        serve_sweep(args)
        return

    if args.gather_count > 0:
        import torch
        table = torch.zeros(1 << 29, dtype=torch.int64, device="cuda")  # 4 GiB
        idx = torch.randint(0, 1 << 29, (args.gather_count,), generator=torch.Generator().manual_seed(1)).cuda()
        out = torch.empty(args.gather_count, dtype=torch.int64, device="cuda")
        for _ in range(5):
            torch.index_select(table, 0, idx, out=out)
        torch.cuda.synchronize()
        log(f"[bench] gathered {args.gather_count} random words 5 times")
        return

    if args.copy_bytes > 0:
        import torch
        src = torch.ones(args.copy_bytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_bytes} bytes 5 times")
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (the library has no multi-GPU path; "
                                   "sharding by pattern is described in the design notes)", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.profile_pass:
        args.steps = args.warmup = 0
        args.no_cpu = True
        args.plain_seconds = 0
        args.serve_probe_rate = 0

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    pool = None if args.no_cpu else start_cpu_pool(threads)

    import torch

    from paper_2404_01585_amd import flexis as fx
    from paper_2404_01585_amd import mining
    from paper_2404_01585_amd.synth import workload_graph

    spec = WORKLOADS[args.workload]
    t = time.perf_counter()
    g = workload_graph(spec["graph"])
    log(f"[bench] graph {spec['graph']}: {g.num_vertices} vertices, {g.num_adj // 2} edges "
        f"({time.perf_counter() - t:.1f} s)")
    torch.cuda.set_device(0)
    ctx = fx.Context(device=0, no_digest=not args.digest, count_cap=args.count_cap,
                     run_index_bytes=-1 if args.no_run_index else 0)
    t = time.perf_counter()
    dg = ctx.load_graph(g)
    log(f"[bench] graph resident on the device ({time.perf_counter() - t:.1f} s)")
    mode = fx.MODE_FULL if args.mode == "full" else fx.MODE_VERDICT
    lams = spec["lams"]
    types = mining.edge_types(g) if "levels" in spec else None
    batches, per_level = [], {}
    for lam in lams:
        t = time.perf_counter()
        cands, pl = build_candidates(dg, g, spec, lam, types=types)
        b = fx.PatternBatch(cands)
        b.sigma = spec["sigma"]
        batches.append((lam, b))
        per_level[str(lam)] = pl
        log(f"[bench] lambda {lam}: candidates {len(cands)} per level {pl} ({time.perf_counter() - t:.1f} s)")

    shape = dict(spec.get("shape") or {})
    for k in SHAPE_KEYS:
        v = getattr(args, k)
        if v is not None:
            shape[k] = v
    tuned = None
    if args.autotune:
        t = time.perf_counter()
        lam0, b0 = batches[-1]
        tuned = dg.autotune(b0, spec["sigma"], lam0, mode, cache_path=args.tune_cache)
        log(f"[bench] autotune {tuned} ({time.perf_counter() - t:.1f} s)")
    else:
        apply_shape(ctx, shape)
    for k in ENGINE_KEYS:
        if getattr(args, k) is not None:
            ctx.set(k, getattr(args, k))
    shape = {k: ctx.get(k) for k in SHAPE_KEYS + ENGINE_KEYS}
    log(f"[bench] launch shape {shape}")

    for w in range(args.warmup):
        lam, b = batches[w % len(batches)]
        dg.support_batch_array(b, spec["sigma"], lam, mode)
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ctx.stats(reset=True)
    npat = 0
    emb = 0
    qms, qsteps, rounds_max, frequent = [], [], 0, 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        lam, b = batches[k % len(batches)]
        res = dg.support_batch_array(b, spec["sigma"], lam, mode)
        npat += len(b)
        ok = (res["embedding_count"] > 0) & (res["count_saturated"] == 0)
        emb += int(res["embedding_count"][ok].sum())
        qms.append(res["device_ms"])
        qsteps.append(res["steps"])
        rounds_max = max(rounds_max, int(res["rounds"].max()) if len(res) else 0)
        frequent += int(res["frequent"].sum())
        log(f"[bench] step {k + 1}/{args.steps} done (lambda {lam}, {len(b)} patterns)")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.stats(reset=True)

    roofline = None
    if not args.no_roofline:
        traffic = traffic_from_profile(os.path.join(ROOT, "paper_2404_01585_amd", "csrc", "fx_kernels.hip"),
                                       args.workload)
        roofline = roofline_pass(ctx, dg, batches, mode, args.roofline_repeats, not args.profile_pass, traffic)
        log(f"[bench] roofline {roofline}")
    if args.profile_pass:
        print(json.dumps({"profile_pass": args.workload, "roofline": roofline, "shape": shape}), flush=True)
        dg.close()
        ctx.close()
        return

    allc = [p for _, b in batches for p in b.patterns]
    alls = [spec["sigma"]] * len(allc)
    alll = [lam for lam, b in batches for _ in b.patterns]
    # the plain form for comparison: one pattern per call, cycling through the batches
    plain = None
    if args.plain_seconds > 0:
        offs = np.cumsum([0] + [len(b) for _, b in batches])
        order = [int(offs[q]) + j for j in range(max(len(b) for _, b in batches))
                 for q in range(len(batches)) if j < len(batches[q][1])]
        t1 = time.perf_counter()
        k = 0
        while k < len(order) and time.perf_counter() - t1 < args.plain_seconds:
            i = order[k]
            dg.support(allc[i], alls[i], alll[i], mode)
            k += 1
        plain = dict(patterns_per_s=round(k / (time.perf_counter() - t1), 3), sample=k)
        log(f"[bench] plain form: {plain}")

    serving = None
    if args.serve_probe_rate > 0:
        gs = g if args.serve_probe_graph == spec["graph"] else workload_graph(args.serve_probe_graph)
        dgs = dg if gs is g else ctx.load_graph(gs)
        queries = serving_queries(gs, args.serve_probe_queries, seed=4)
        with fx.Server(dgs, no_digest=not args.digest, step_candidates=args.serve_step) as srv:
            run_served(srv, tuple(x[:100] for x in queries), args.serve_probe_rate, fx.MODE_VERDICT, seed=99)
            served, _ = run_served(srv, queries, args.serve_probe_rate, fx.MODE_VERDICT, seed=7)
        fifo, _ = run_fifo(dgs, queries, args.serve_probe_rate, fx.MODE_VERDICT, seed=7)
        if dgs is not dg:
            dgs.close()
        serving = dict(graph=args.serve_probe_graph, rate_qps=args.serve_probe_rate,
                       queries=args.serve_probe_queries, mode="verdict", served=served, fifo_one_per_call=fifo)
        log(f"[bench] serving probe: {serving}")

    cpu = None
    if not args.no_cpu:
        log(f"[bench] cpu baseline: oracle on {threads} processes for ~{args.cpu_seconds} s")
        cpu = cpu_baseline(pool, threads, g, allc, alls, alll, args.cpu_seconds)
        log(f"[bench] cpu baseline: {cpu}")

    qms = np.concatenate(qms) if qms else np.zeros(1)
    qsteps = np.concatenate(qsteps) if qsteps else np.zeros(1, dtype=np.int64)
    line = {
        "metric": "candidate patterns/s (support queries, FULL mode) at 1 GPU",
        "value": round(npat / dt, 3) if dt > 0 else None,
        "unit": "patterns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / max(args.steps, 1), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": spec["desc"],
                   "patterns_per_lambda": {str(lam): len(b) for lam, b in batches},
                   "patterns_per_level": per_level, "sigma": spec["sigma"], "lambdas": lams,
                   "mode": args.mode, "count_cap": ctx.count_cap, "digest": bool(args.digest),
                   "run_index": not args.no_run_index,
                   "form": "batched (all candidates of the batch in flight, one segment each per device step)",
                   "shape": shape, "tuned": tuned},
        "embeddings_per_s": round(emb / dt, 1) if dt > 0 else None,
        "frequent_per_step": round(frequent / max(args.steps, 1), 1),
        "query_device_ms_p50": round(float(np.percentile(qms, 50)), 4),
        "query_device_ms_p99": round(float(np.percentile(qms, 99)), 4),
        "query_steps_p50_p99_max": [int(np.percentile(qsteps, 50)), int(np.percentile(qsteps, 99)),
                                    int(qsteps.max())],
        "greedy_rounds_max": rounds_max,
        "syncs_per_step": st["syncs"] / max(args.steps, 1),
        "reoffered_candidates_per_step": st["reoffered"] / max(args.steps, 1),
        "stack_promotions_per_step": st["promotions"] / max(args.steps, 1),
        "host_ms_per_step": round(st["host_ms"] / max(args.steps, 1), 3),
        "device_wait_ms_per_step": round(st["wait_ms"] / max(args.steps, 1), 3),
        "device_steps_per_step": st["steps"] / max(args.steps, 1),
        "chained_steps_per_step": st["chain_steps"] / max(args.steps, 1),
        "chains_per_step": st["chains"] / max(args.steps, 1),
        "probed_candidates_per_step": st["probed"] / max(args.steps, 1),
        "plain_form": plain,
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    dg.close()
    ctx.close()


if __name__ == "__main__":
    main()
