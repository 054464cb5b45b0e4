"""Benchmark of the (k,h)-core hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--stages ...]

Workload: Chung-Lu power-law graph, n = 1,000,000, m = 10,000,000 undirected
edges, degree exponent 2.1 (seed 1, int32 CSR), resident in HBM before the
timed region.  One step runs the selected stages of the hot path at h = 2
and h = 3:

  hdeg     all-vertex exact h-degrees (bit-parallel multi-source BFS)
  exact    ExactCore: h-degrees + frontier-driven bulk peel + densest core
  sampled  Core (Alg. 4, eps = 0.5, delta = 0.05): ranks, sample-list union
           over h hops, estimate, bulk peel with lazy update, densest core

Metric: edges traversed per second (the arcs a per-source bounded BFS
inspects, summed over every h-degree evaluation the step performs) over the
whole step time.  The JSON line also carries the pull kernel's roofline
(HIP-event timed inside the library, algorithmic bytes counted by the
kernel) and the CPU oracle's rate on a bounded sample of sources.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
WORKLOAD = "chung_lu n=1000000 m=10000000 gamma=2.1 seed=1"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(g, hs, budget_s: float):
    """The oracle's per-source BFS h-degrees on a seeded sample of sources,
    single thread, about budget_s seconds per h."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(12345)
    order = rng.permutation(g.n).astype(np.int32)
    te_tot, t_tot, nsrc = 0, 0.0, 0
    per_h = {}
    for h in hs:
        te_h, t_h, k = 0, 0.0, 0
        while t_h < budget_s and k < g.n:
            chunk = order[k:k + 32]
            t0 = time.perf_counter()
            _, te = oracle.hdeg_list(g, h, chunk, with_te=True)
            t_h += time.perf_counter() - t0
            te_h += te
            k += chunk.size
        per_h[h] = {"sources": k, "te": te_h, "seconds": t_h}
        te_tot += te_h
        t_tot += t_h
        nsrc += k
    return {"value": te_tot / t_tot, "unit": "edges_traversed/s", "cores": 1, "kind": "oracle",
            "sample": f"per-source BFS h-degrees of {nsrc} seeded random sources (h in {list(hs)}), "
                      f"about {budget_s:.0f} s per h, single thread", "per_h": per_h}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--stages", default="hdeg", help="comma list of hdeg,exact,sampled")
    ap.add_argument("--hs", default="2,3")
    ap.add_argument("--cpu-budget", type=float, default=8.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    import paper_2112_06154_amd as kh

    stages = [s for s in args.stages.split(",") if s]
    hs = [int(x) for x in args.hs.split(",")]
    t0 = time.time()
    g = gg.workload("cl1m")
    log(f"graph {WORKLOAD}: generated in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    ctx = kh.Context(0)
    G = kh.Graph.from_gg(ctx, g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()

    if args.copy_calib:
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step(record):
        te = 0
        for h in hs:
            if "hdeg" in stages:
                t = time.perf_counter()
                _, e = kh.hdeg(G, h, out=out)
                torch.cuda.synchronize()
                record.setdefault(f"hdeg_h{h}_s", []).append(time.perf_counter() - t)
                te += e
            if "exact" in stages:
                t = time.perf_counter()
                _, res = kh.core(G, h, out=out, dense=True)
                torch.cuda.synchronize()
                record.setdefault(f"exact_h{h}_s", []).append(time.perf_counter() - t)
                record[f"exact_h{h}_rounds"] = res["rounds"]
                te += res["edges_traversed"]
            if "sampled" in stages:
                t = time.perf_counter()
                _, res = kh.core(G, h, epsilon=0.5, delta=0.05, seed=1, out=out, dense=True)
                torch.cuda.synchronize()
                record.setdefault(f"sampled_h{h}_s", []).append(time.perf_counter() - t)
                record[f"sampled_h{h}_rounds"] = res["rounds"]
                record[f"sampled_h{h}_max_core"] = res["max_core"]
        return te

    warm = {}
    for i in range(args.warmup):
        step(warm)
        log(f"warmup {i + 1}/{args.warmup} done")
    rec = {}
    ctx.profile(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    te_total = 0
    for i in range(args.steps):
        te_total += step(rec)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = ctx.profile_read()
    ctx.profile(False)

    value = te_total / elapsed
    pull_ms = prof["ms"]
    achieved = (prof["alg_bytes"] / (pull_ms * 1e-3)) / 1e9 if pull_ms > 0 else 0.0
    roof = {
        "kernel": "k_ms_pull<16> (h-degree pull hop)",
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "launches": prof["launches"],
        "avg_launch_ms": round(pull_ms / max(prof["launches"], 1), 4),
        "alg_bytes_per_launch": prof["alg_bytes"] // max(prof["launches"], 1),
        "gather_bytes_per_launch": prof["gather_bytes"] // max(prof["launches"], 1),
        "gather_gbs": round((prof["gather_bytes"] / (pull_ms * 1e-3)) / 1e9, 2) if pull_ms > 0 else 0.0,
    }
    line = {
        "metric": "(k,h)-core edges-traversed/sec + %HBM roofline at h=2,3",
        "value": value, "unit": "edges_traversed/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": WORKLOAD, "h": hs, "stages": stages, "epsilon": 0.5, "delta": 0.05},
        "roofline": roof,
        "stage_seconds": {k: v for k, v in rec.items()},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(g, hs, args.cpu_budget)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
