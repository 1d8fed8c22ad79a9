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
    "er1k-l4": dict(graph="er1k", sigma=20, lam=1.0, levels=4,
                    desc="Erdos-Renyi 1K vertices / 4K edges, 5 uniform vertex labels, 1 edge label; all "
                         "candidates of mining levels 1-4 at sigma=20, lambda=1.0"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_candidates(dg, g, spec):
    """Candidate batch: every candidate of the first `levels` mining levels.
    The level-wise loop itself runs here (untimed), with verdicts from the
    device path."""
    from paper_2404_01585_amd import flexis as fx
    from paper_2404_01585_amd import mining

    def evaluate(ps, sigma, lam):
        return dg.support_batch(ps, [sigma] * len(ps), [lam] * len(ps), fx.MODE_VERDICT)

    res = mining.mine(g, spec["sigma"], spec["lam"], spec["levels"], evaluate, tau_fn=fx.tau)
    cands = [p for lvl in res["levels"] for p in lvl]
    return cands, [len(l) for l in res["levels"]]


def traffic_from_profile(kernel_src: str):
    """HBM traffic per probe launch from the committed PMC summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_probe_cl100k-l2.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sha256") != hashlib.sha256(open(kernel_src, "rb").read()).hexdigest():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(g, cands, spec, seconds: float, threads: int):
    """The oracle (untuned) on the host cores: FULL-mode queries over a prefix
    of the same batch, spread over a thread pool, bounded to ~`seconds`."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O

    OG = O.OracleGraph.of(g)
    pats = [O.OraclePattern.of(p) for p in cands]
    t0 = time.perf_counter()
    deadline = t0 + seconds
    done = 0
    idx = 0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        while idx < len(pats) and time.perf_counter() < deadline:
            chunk = pats[idx:idx + 4 * threads]
            list(ex.map(lambda p: O.query(OG, p, spec["sigma"], spec["lam"], O.FULL), chunk))
            idx += len(chunk)
            done += len(chunk)
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="patterns/s", cores=threads, kind="oracle",
                sample=f"first {done} of {len(pats)} candidates of the same batch, FULL mode "
                       f"(support + count + digest), {dt:.1f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl100k-l2", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="full", choices=["full", "verdict"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--digest", action="store_true",
                    help="also hash every embedding (FULL-mode digest); counts are exact either way")
    ap.add_argument("--plain-seconds", type=float, default=5.0,
                    help="time the one-pattern-per-call form on a prefix of the batch for this long")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="calibration only: copy a buffer of this many bytes 5 times with torch and exit "
                         "(a plain copy kernel of known size for the PMC traffic factors)")
    args = ap.parse_args()

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
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is described in the design "
                                   "notes but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2404_01585_amd import flexis as fx
    from paper_2404_01585_amd.synth import workload_graph

    spec = WORKLOADS[args.workload]
    t = time.perf_counter()
    g = workload_graph(spec["graph"])
    log(f"[bench] graph {spec['graph']}: {g.num_vertices} vertices, {g.num_adj // 2} edges "
        f"({time.perf_counter() - t:.1f} s)")
    torch.cuda.set_device(0)
    ctx = fx.Context(device=0, kernel_timing=not args.no_timing, no_digest=not args.digest)
    dg = ctx.load_graph(g)
    t = time.perf_counter()
    cands, per_level = build_candidates(dg, g, spec)
    log(f"[bench] candidates {len(cands)} per level {per_level} ({time.perf_counter() - t:.1f} s)")
    mode = fx.MODE_FULL if args.mode == "full" else fx.MODE_VERDICT
    sig = [spec["sigma"]] * len(cands)
    lam = [spec["lam"]] * len(cands)
    batch = fx.PatternBatch(cands)

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
                                                                  "fx_kernels.hip")),
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

    cpu = None
    if not args.no_cpu:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"[bench] cpu baseline: oracle on {threads} threads for ~{args.cpu_seconds} s")
        cpu = cpu_baseline(g, cands, spec, args.cpu_seconds, threads)

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
                   "form": "batched (all candidates of the batch in flight, one segment each per step)"},
        "embeddings_per_s": round(emb * args.steps / dt, 1),
        "frequent": frequent,
        "query_device_ms_p50": round(float(np.percentile(qms, 50)), 4),
        "query_device_ms_p99": round(float(np.percentile(qms, 99)), 4),
        "query_steps_p50_p99_max": [int(np.percentile(results["steps"], 50)), int(np.percentile(results["steps"], 99)),
                                    int(results["steps"].max())],
        "greedy_rounds_max": int(results["rounds"].max()),
        "syncs_per_step": st["syncs"] / args.steps,
        "device_steps_per_step": st["steps"] / args.steps,
        "plain_form": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    dg.close()
    ctx.close()


if __name__ == "__main__":
    main()
