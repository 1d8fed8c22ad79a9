#!/usr/bin/env python3
"""Support-counting throughput on one MI355X.

A step is one pass of the whole hot path over one batch of candidate
patterns: for every pattern, enumerate its embeddings, take the greedy
maximal independent set, compare it with tau, and count and hash the
embeddings (FULL mode), all through the C ABI of libflexis.so.

Default workload ("cl100k-l2"): Chung-Lu graph with 100,000 vertices and
500,000 edges (degree exponent 2.1, structural cutoff sqrt(2m)), 20 vertex
labels Zipf(1.2), 3 edge labels uniform; the batch is every candidate of the
first two levels of the mining loop (Algorithm 1) at sigma = 200,
lambda = 1.0 -- all labeled edges and all one-edge extensions of the
frequent ones.  Inputs are synthetic and seeded; the graph is resident in
HBM before the timed region.

Prints one JSON line (metric, value = patterns/s, roofline of the dominant
kernel from live HIP-event timing, and the CPU oracle's rate on a bounded
sample of the same batch).
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

WORKLOADS = {
    "cl100k-l2": dict(graph="cl100k", sigma=200, lam=1.0, levels=2,
                      desc="Chung-Lu 100K vertices / 500K edges (gamma 2.1), 20 Zipf(1.2) vertex labels, "
                           "3 edge labels; all candidates of mining levels 1-2 at sigma=200, lambda=1.0"),
    "cl100k-l3": dict(graph="cl100k", sigma=200, lam=1.0, levels=3,
                      desc="Chung-Lu 100K vertices / 500K edges (gamma 2.1), 20 Zipf(1.2) vertex labels, "
                           "3 edge labels; all candidates of mining levels 1-3 at sigma=200, lambda=1.0"),
    "cl100k-l2-l03": dict(graph="cl100k", sigma=200, lam=0.3, levels=2,
                          desc="as cl100k-l2 with lambda=0.3"),
    "cl1m-s2000": dict(graph="cl1m", sigma=200, lam=1.0, sample=dict(count=2000, seed=33, kmin=3, kmax=7),
                       desc="Chung-Lu 1M vertices / 8M edges (gamma 2.3), 30 Zipf(1.0) vertex labels, 1 edge "
                            "label; 2,000 patterns of 3-7 vertices (trees, cycles, trees plus a chord) sampled "
                            "as connected subgraphs of the graph, sigma=200, lambda=1.0"),
    "rmat22-l2": dict(graph="rmat22", sigma=2000, lam=1.0, levels=2,
                      desc="R-MAT scale 22 (4,194,304 vertices, 40M edges, a,b,c = 0.57,0.19,0.19), 50 Zipf(1.1) "
                           "vertex labels, 4 edge labels, int64 offsets; all candidates of mining levels 1-2 at "
                           "sigma=2000, lambda=1.0"),
    "cl100k-v4": dict(graph="cl100k", sigma=200, lam=1.0, vertices=4,
                      desc="Chung-Lu 100K vertices / 500K edges (gamma 2.1), 20 Zipf(1.2) vertex labels, "
                           "3 edge labels; all candidates of the merge generator (levels by vertex count) up to "
                           "4 vertices at sigma=200, lambda=1.0"),
    "er1k-l4": dict(graph="er1k", sigma=20, lam=1.0, levels=4,
                    desc="Erdos-Renyi 1K vertices / 4K edges, 5 uniform vertex labels, 1 edge label; all "
                         "candidates of mining levels 1-4 at sigma=20, lambda=1.0"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_candidates(dg, g, spec):
    """Candidate batch: patterns sampled from the graph, or every candidate
    of the first `levels` mining levels (the level-wise loop itself runs here,
    untimed, with verdicts from the device path)."""
    from paper_2404_01585_amd import flexis as fx
    from paper_2404_01585_amd import mining
    from paper_2404_01585_amd.synth import sample_patterns

    if "sample" in spec:
        sm = spec["sample"]
        cands = sample_patterns(g, sm["count"], seed=sm["seed"], kmin=sm["kmin"], kmax=sm["kmax"])
        return cands, [len(cands)]

    if "vertices" in spec:  # Algorithm 1 with the merge generator (Algorithms 2-4)
        from paper_2404_01585_amd import generate

        def ev(ps, sigma, lam):
            return dg.support_batch(ps, [sigma] * len(ps), [lam] * len(ps), fx.MODE_VERDICT)

        res = generate.mine_by_vertices(g, spec["sigma"], spec["lam"], spec["vertices"], ev, fx.tau)
        cands = [p for lvl in res["levels"] for p in lvl]
        return cands, [len(l) for l in res["levels"]]

    def evaluate(ps, sigma, lam):
        return dg.support_batch(ps, [sigma] * len(ps), [lam] * len(ps), fx.MODE_VERDICT)

    res = mining.mine(g, spec["sigma"], spec["lam"], spec["levels"], evaluate, tau_fn=fx.tau)
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


def _cpu_task(args):
    """Worker of the CPU baseline: one FULL-mode oracle query.  The graph and
    the batch are read once per worker from the file the parent wrote."""
    path, i = args
    from oracle import oracle as O

    if _CPU.get("path") != path:
        z = np.load(path)
        _CPU.update(path=path, g=O.OracleGraph(z["row_ptr"], z["col"], z["vlabel"], z["elabel"]),
                    pats=[O.OraclePattern(p["vlabel"], p["edges"], p["elabel"])
                          for p in json.loads(str(z["patterns"]))],
                    sigma=int(z["sigma"]), lam=float(z["lam"]))
    O.query(_CPU["g"], _CPU["pats"][i], _CPU["sigma"], _CPU["lam"], O.FULL)
    return i


def start_cpu_pool(threads: int):
    """Worker processes of the CPU baseline, started before this process
    touches the GPU (they never do)."""
    import multiprocessing as mp

    return mp.get_context("spawn").Pool(threads)


def cpu_baseline(pool, threads: int, g, cands, spec, seconds: float):
    """The oracle (untuned) on the host cores: FULL-mode queries over the
    batch in order, one per worker process, for about `seconds`; the rate is
    the queries finished by then over the wall time (queries still running
    at the deadline are not counted)."""
    import tempfile

    fd, path = tempfile.mkstemp(suffix=".npz", prefix="fx_cpu_")
    os.close(fd)
    try:
        pats = [dict(vlabel=list(map(int, p.vlabel)), edges=[list(map(int, e)) for e in p.edges],
                     elabel=list(map(int, p.elabel))) for p in cands]
        with open(path, "wb") as f:
            np.savez(f, row_ptr=g.row_ptr, col=g.col, vlabel=g.vlabel, elabel=g.elabel,
                     patterns=np.array(json.dumps(pats)), sigma=spec["sigma"], lam=spec["lam"])
        t0 = time.perf_counter()
        deadline = t0 + seconds
        done = 0
        it = pool.imap_unordered(_cpu_task, [(path, i) for i in range(len(cands))])
        while True:
            left = deadline - time.perf_counter()
            if left <= 0:
                break
            try:
                it.next(timeout=left)
            except StopIteration:
                break
            except __import__("multiprocessing").TimeoutError:
                break
            done += 1
        dt = time.perf_counter() - t0
    finally:
        pool.terminate()
        pool.join()
        os.unlink(path)
    return dict(value=done / dt, unit="patterns/s", cores=threads, kind="oracle",
                sample=f"{done} of {len(cands)} candidates of the same batch finished in {dt:.1f} s wall, "
                       f"taken in batch order, FULL mode (support + count + digest), one process per core")


def serving_queries(g, count: int, seed: int):
    """Support queries of the serving workload: patterns of 3-8 vertices
    sampled from the graph, sigma log-uniform in [50, 5000], lambda uniform in
    {0.1, 0.5, 1.0}."""
    import numpy as np

    from paper_2404_01585_amd.synth import sample_patterns

    rng = np.random.default_rng(seed)
    pats = sample_patterns(g, count, seed=seed, kmin=3, kmax=8)
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
    log(f"[serve] {n} submitted at {rate} q/s")
    res = []
    for k, t in enumerate(tickets):
        res.append(srv.wait(t))
        if (k + 1) % 250 == 0:
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
        if (i + 1) % 100 == 0:
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

    g = workload_graph("cl100k")
    torch.cuda.set_device(0)
    ctx = fx.Context(device=0, no_digest=True, count_cap=args.serve_count_cap)
    dg = ctx.load_graph(g)
    queries = serving_queries(g, args.serve_queries, seed=4)
    log(f"[serve] {len(queries[0])} queries sampled")
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
            "config": {"workload": "cl100k-serve: Chung-Lu 100K vertices / 500K edges resident; Poisson arrivals; "
                                   "patterns of 3-8 vertices sampled from the graph; sigma log-uniform [50, 5000]; "
                                   "lambda in {0.1, 0.5, 1.0}", "queries_per_rate_verdict": args.serve_queries,
                       "queries_per_rate_full": args.serve_full_queries, "count_cap_full": args.serve_count_cap,
                       "step_candidates": args.serve_step},
            "rates": out}
    print(json.dumps(line), flush=True)
    dg.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl100k-l2", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="full", choices=["full", "verdict"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--count-cap", type=int, default=0, help="embedding count cap (0: 2^62)")
    ap.add_argument("--no-run-index", action="store_true",
                    help="no label-run index: candidate runs and edge tests by binary search in the rows")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (untimed) before the timed steps")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: a later run with the same file reuses the same launch shape")
    ap.add_argument("--digest", action="store_true",
                    help="also hash every embedding (FULL-mode digest); counts are exact either way")
    ap.add_argument("--plain-seconds", type=float, default=5.0,
                    help="time the one-pattern-per-call form on a prefix of the batch for this long")
    ap.add_argument("--serve", action="store_true", help="serving sweep (Poisson arrivals) instead of the batch")
    ap.add_argument("--serve-rates", default="100,300,1000,3000,5000")
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--serve-full-rates", default="100,1000")
    ap.add_argument("--serve-full-queries", type=int, default=300)
    ap.add_argument("--serve-count-cap", type=int, default=10 ** 9)
    ap.add_argument("--serve-step", type=int, default=1 << 22, help="candidates per device step of the server")
    ap.add_argument("--no-fifo", action="store_true")
    ap.add_argument("--serve-probe-rate", type=float, default=1000.0,
                    help="rate of the short serving probe in the default run (0: skip)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="calibration only: copy a buffer of this many bytes 5 times with torch and exit "
                         "(a plain copy kernel of known size for the PMC traffic factors)")
    args = ap.parse_args()

    if args.serve:
        serve_sweep(args)
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

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    pool = None if args.no_cpu else start_cpu_pool(threads)

    import torch

    from paper_2404_01585_amd import flexis as fx
    from paper_2404_01585_amd.synth import workload_graph

    spec = WORKLOADS[args.workload]
    t = time.perf_counter()
    g = workload_graph(spec["graph"])
    log(f"[bench] graph {spec['graph']}: {g.num_vertices} vertices, {g.num_adj // 2} edges "
        f"({time.perf_counter() - t:.1f} s)")
    torch.cuda.set_device(0)
    ctx = fx.Context(device=0, kernel_timing=not args.no_timing, no_digest=not args.digest,
                     count_cap=args.count_cap, run_index_bytes=-1 if args.no_run_index else 0)
    dg = ctx.load_graph(g)
    t = time.perf_counter()
    cands, per_level = build_candidates(dg, g, spec)
    log(f"[bench] candidates {len(cands)} per level {per_level} ({time.perf_counter() - t:.1f} s)")
    mode = fx.MODE_FULL if args.mode == "full" else fx.MODE_VERDICT
    sig = [spec["sigma"]] * len(cands)
    lam = [spec["lam"]] * len(cands)
    batch = fx.PatternBatch(cands)

    tuned = None
    if not args.no_tune:
        t = time.perf_counter()
        tuned = dg.autotune(batch, spec["sigma"], spec["lam"], mode, cache_path=args.tune_cache)
        log(f"[bench] autotune {tuned} ({time.perf_counter() - t:.1f} s)")
    for w in range(args.warmup):
        dg.support_batch_array(batch, spec["sigma"], spec["lam"], mode)
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ctx.stats(reset=True)
    results = None
    t0 = time.perf_counter()
    for k in range(args.steps):
        results = dg.support_batch_array(batch, spec["sigma"], spec["lam"], mode)
        log(f"[bench] step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.stats()

    P = len(cands)
    value = P * args.steps / dt
    ok = (results["embedding_count"] > 0) & (results["count_saturated"] == 0)
    emb = int(results["embedding_count"][ok].sum())
    qms = results["device_ms"]
    frequent = int(results["frequent"].sum())

    roofline = None
    if st["probe_launches"] and st["probe_ms"] > 0:
        avg_ms = st["probe_ms"] / st["probe_launches"]
        bytes_per_launch = st["probe_alg_bytes"] / st["probe_launches"]
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        roofline = dict(bound="hbm", achieved=round(achieved, 3), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 6),
                        traffic=traffic_from_profile(os.path.join(ROOT, "paper_2404_01585_amd", "csrc",
                                                                  "fx_kernels.hip"), args.workload),
                        kernel="k_probe", avg_launch_us=round(avg_ms * 1e3, 3),
                        alg_bytes_per_launch=round(bytes_per_launch, 1), launches=st["probe_launches"],
                        kernel_ms_share=dict(probe=round(st["probe_ms"], 3), scatter=round(st["scatter_ms"], 3),
                                             greedy=round(st["greedy_ms"], 3)))

    # the plain form for comparison: one pattern per call, on a prefix of the batch
    plain = None
    if args.plain_seconds > 0:
        t1 = time.perf_counter()
        k = 0
        while k < P and time.perf_counter() - t1 < args.plain_seconds:
            dg.support(cands[k], sig[k], lam[k], mode)
            k += 1
        plain = dict(patterns_per_s=round(k / (time.perf_counter() - t1), 3), sample=k)
        log(f"[bench] plain form: {plain}")

    serving = None
    if args.serve_probe_rate > 0:
        queries = serving_queries(g, 1000, seed=4)
        with fx.Server(dg, no_digest=not args.digest, step_candidates=args.serve_step) as srv:
            run_served(srv, tuple(x[:100] for x in queries), 1000.0, fx.MODE_VERDICT, seed=99)
            served, _ = run_served(srv, queries, args.serve_probe_rate, fx.MODE_VERDICT, seed=7)
        fifo, _ = run_fifo(dg, queries, args.serve_probe_rate, fx.MODE_VERDICT, seed=7)
        serving = dict(rate_qps=args.serve_probe_rate, mode="verdict", served=served, fifo_one_per_call=fifo)
        log(f"[bench] serving probe: {serving}")

    cpu = None
    if not args.no_cpu:
        log(f"[bench] cpu baseline: oracle on {threads} processes for ~{args.cpu_seconds} s")
        cpu = cpu_baseline(pool, threads, g, cands, spec, args.cpu_seconds)

    line = {
        "metric": "candidate patterns/s (support queries, FULL mode) at 1 GPU",
        "value": round(value, 3),
        "unit": "patterns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": spec["desc"], "patterns": P,
                   "patterns_per_level": per_level, "sigma": spec["sigma"], "lambda": spec["lam"],
                   "mode": args.mode, "count_cap": ctx.count_cap, "digest": bool(args.digest),
                   "run_index": not args.no_run_index,
                   "form": "batched (all candidates of the batch in flight, one segment each per step)",
                   "tuned": tuned},
        "embeddings_per_s": round(emb * args.steps / dt, 1),
        "frequent": frequent,
        "query_device_ms_p50": round(float(np.percentile(qms, 50)), 4),
        "query_device_ms_p99": round(float(np.percentile(qms, 99)), 4),
        "query_steps_p50_p99_max": [int(np.percentile(results["steps"], 50)), int(np.percentile(results["steps"], 99)),
                                    int(results["steps"].max())],
        "greedy_rounds_max": int(results["rounds"].max()),
        "syncs_per_step": st["syncs"] / args.steps,
        "reoffered_candidates_per_step": st["reoffered"] / args.steps,
        "stack_promotions_per_step": st["promotions"] / args.steps,
        "host_ms_per_step": round(st["host_ms"] / args.steps, 3),
        "device_wait_ms_per_step": round(st["wait_ms"] / args.steps, 3),
        "device_steps_per_step": st["steps"] / args.steps,
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
