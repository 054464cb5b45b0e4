"""Benchmark of the (k,h)-core hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget-s S] [...]

Workload: Chung-Lu power-law graph, n = 1,000,000, m = 10,000,000 undirected
edges, degree exponent 2.1 (seed 1, int32 CSR), resident in HBM before the
timed region.  One step runs the whole hot path at h = 2 and h = 3 (--hs):

  exact    ExactCore: h-degrees by bit-parallel bounded BFS, frontier-driven
           bulk peel, densest core level (pruning variant)
  sampled  Core (Alg. 4, eps = 0.5, delta = 0.05): ranks, sample-list union
           over h hops, estimate, bulk peel with lazy update, densest-core
           estimate (Alg. 7, core levels, pruning variant); the top level is
           initialised lazily at the h listed in --lazy-hs (3 by default)

Metric: edges traversed per second of ExactCore, from the library's own count
(kh_result.edges_traversed: for every h-degree the peel evaluates, the arcs a
per-source bounded BFS inspects), summed over the exact decompositions of the
timed steps and divided by their wall time.  The sampled path traverses no
BFS edges; its rate is reported beside it as sample-list elements merged per
second.  ms_per_step is the wall time of the whole step.

The run keeps to a wall-clock budget (--budget-s, counted from the start of
the process): warmup and timed steps are cut to what fits, at least one timed
step, and the JSON line reports the counts actually run.  Timed steps come
first: a warmup step beyond the first runs only if every requested timed step
still fits after it.  The JSON line also
carries the roofline of the dominant instrumented kernel (HIP events on its
launch stream inside the library, algorithmic bytes counted by the kernel) and
the CPU oracle's rate on a bounded sample of sources, over all host cores.
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
KERNEL_SRC = {0: "paper_2112_06154_amd/csrc/kh_msbfs.hip", 1: "paper_2112_06154_amd/csrc/kh_union.hip",
              2: "paper_2112_06154_amd/csrc/kh_graph.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")


def source_hash(k):
    import hashlib
    with open(os.path.join(ROOT, KERNEL_SRC[k]), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(k, stages, hs):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE counter
    runs, if they were taken on this kernel source and workload; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(str(k))
    if not e or e.get("source_sha256_16") != source_hash(k):
        return None
    if e.get("stage") != stages or e.get("h") != hs:
        return None
    return e.get("bytes_per_launch")


# the dispatches counted as one launch of a reported kernel (the union's hubs
# are merged by a second, wider variant inside the same timed launch)
KERNEL_NAMES = {0: ["k_ms_pull<16>", "k_ms_pull<8>", "k_ms_pull<4>", "k_ms_pull<2>", "k_ms_pull<1>"],
                1: ["k_union<256>", "k_union<64>", "k_union<1024>", "k_hub_units", "k_union_merge<256>"],
                2: ["k_rbfs_hop"]}
# FETCH_SIZE reads 524,317 KiB for the 1 GiB read by the add kernel of
# --copy-calib, WRITE_SIZE 1,048,576 KiB for its 1 GiB write
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def pmc_summarize(fetch_dir, write_dir, stages, hs, out_path=None):
    """Per-launch HBM bytes of the two reported kernels from rocprofv3
    counter_collection.csv files of a FETCH_SIZE run and a WRITE_SIZE run of
    the same command (KiB per dispatch, scaled by the copy calibration), plus
    the calibration kernels' readings; written to profiles/traffic_counters.json."""
    import csv
    import glob

    def per_kernel(d, counter):
        agg = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row.get("Counter_Name") != counter:
                        continue
                    name = row["Kernel_Name"].split("(")[0].replace("void ", "").replace("kh::", "")
                    a = agg.setdefault(name, [0, 0.0])
                    a[0] += 1
                    a[1] += float(row["Counter_Value"])
        return agg

    fe, wr = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    out = {"scale": {"FETCH_SIZE": FETCH_SCALE, "WRITE_SIZE": WRITE_SCALE},
           "calibration": {k: {"fetch_kib": v[1] / v[0], "write_kib": wr[k][1] / wr[k][0] if k in wr else None}
                           for k, v in fe.items() if "at::native" in k}}
    for k, names in KERNEL_NAMES.items():
        first = names[0]
        if first not in fe or first not in wr:
            continue
        # one timed launch = one dispatch of the first variant (the union), or
        # of any variant (the pull kernel's widths)
        launches = sum(fe[nm][0] for nm in names if nm in fe) if k == 0 else fe[first][0]
        f_kib = sum(fe[nm][1] for nm in names if nm in fe) / launches
        w_kib = sum(wr[nm][1] for nm in names if nm in wr) / launches
        out[str(k)] = {"kernels": names, "source_sha256_16": source_hash(k), "stage": stages, "h": hs,
                       "launches": launches, "fetch_kib_per_launch": f_kib, "write_kib_per_launch": w_kib,
                       "bytes_per_launch": int(1024 * (FETCH_SCALE * f_kib + WRITE_SCALE * w_kib))}
    with open(out_path or TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def trace_hops(path):
    """Mask-BFS hop durations of the exact peel from a rocprofv3 kernel_trace.csv
    (--kernel-trace with k_rbfs_hop and k_select_commit included): dispatches
    are numbered by their hop within the round (count since the round's
    k_select_commit) and summed per hop and per duration bucket."""
    import collections
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            nm = r["Kernel_Name"]
            kind = "hop" if "k_rbfs_hop" in nm else ("sel" if "k_select_commit" in nm else None)
            if kind:
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), kind))
    rows.sort()
    by_hop = collections.defaultdict(lambda: [0, 0])
    edges = [5e3, 1e4, 2e4, 5e4, 1e5, 2e5, 5e5, 1e6, float("inf")]
    buckets = collections.defaultdict(lambda: [0, 0])
    hop = 0
    for s0, e0, kind in rows:
        if kind == "sel":
            hop = 0
            continue
        hop += 1
        d = e0 - s0
        by_hop[hop][0] += 1
        by_hop[hop][1] += d
        b = next(x for x in edges if d < x)
        buckets[b][0] += 1
        buckets[b][1] += d
    out = {"hops": {h: {"dispatches": c, "seconds": t / 1e9, "avg_us": t / c / 1e3} for h, (c, t) in by_hop.items()},
           "buckets_us": {("<%g" % (b / 1e3)): {"dispatches": c, "seconds": t / 1e9} for b, (c, t) in buckets.items()}}
    print(json.dumps(out, indent=1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """(threads usable by this process, CPU model) of the host."""
    try:
        cores = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def cpu_baseline(g, hs, budget_s: float, max_threads: int = 16):
    """The oracle's per-source BFS h-degrees on a seeded sample of sources, in
    threads over disjoint source chunks (the oracle is plain C called through
    ctypes, which releases the interpreter lock), about budget_s seconds of
    wall time per h.  Rate = edges traversed / wall time."""
    import concurrent.futures
    import threading

    import numpy as np

    import oracle
    oracle.lib()
    cores, model = host_cpu()
    threads = max(1, min(cores, max_threads))
    rng = np.random.default_rng(12345)
    order = rng.permutation(g.n).astype(np.int32)
    per_h = {}
    te_tot, t_tot, nsrc = 0, 0.0, 0
    for h in hs:
        lock = threading.Lock()
        state = {"next": 0, "te": 0, "src": 0}
        chunk = 256 if h <= 2 else 16  # sources per oracle call (each call sets up an n-sized workspace)
        t0 = time.perf_counter()
        deadline = t0 + budget_s

        def worker():
            while time.perf_counter() < deadline:
                with lock:
                    k = state["next"]
                    if k >= g.n:
                        return
                    state["next"] = k + chunk
                src = order[k:k + chunk]
                _, te = oracle.hdeg_list(g, h, src, with_te=True)
                with lock:
                    state["te"] += te
                    state["src"] += src.size

        with concurrent.futures.ThreadPoolExecutor(threads) as ex:
            for f in [ex.submit(worker) for _ in range(threads)]:
                f.result()
        dt = time.perf_counter() - t0
        per_h[h] = {"sources": state["src"], "te": state["te"], "seconds": round(dt, 3)}
        te_tot += state["te"]
        t_tot += dt
        nsrc += state["src"]
        log(f"cpu baseline h={h}: {state['src']} sources, {state['te'] / dt:.3e} edges traversed/s")
    return {"value": te_tot / t_tot, "unit": "edges_traversed/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "host_threads": cores,
            "sample": f"per-source BFS h-degrees (plain C oracle) of {nsrc} seeded random sources of the same "
                      f"graph, h in {list(hs)}, about {budget_s:.0f} s of wall time per h on {threads} threads",
            "per_h": per_h}


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def bench_batch(kh, ctx, args):
    """Batch workload: many graphs of uneven size (n log-uniform on [100, 50000],
    half Erdos-Renyi with average degree 6, half Barabasi-Albert with 3 edges
    per new vertex), exact (k,h)-cores of all of them by kh_core_batch, against
    kh_core looped over a seeded sample of them (extrapolated)."""
    import numpy as np
    import torch

    import graphgen as gg
    t0 = time.time()
    gs = gg.batch_workload(count=args.batch_count)
    log(f"batch workload: {len(gs)} graphs, {sum(g.n for g in gs)} vertices, generated in {time.time() - t0:.1f}s")
    Gs = [kh.Graph.from_gg(ctx, g) for g in gs]
    torch.cuda.synchronize()
    out = {"graphs": len(gs), "vertices": int(sum(g.n for g in gs)), "edges": int(sum(g.col.size for g in gs) // 2)}
    rng = np.random.default_rng(7)
    half = len(gs) // 2
    sample = sorted(rng.choice(half, args.batch_loop_sample // 2, replace=False).tolist() +
                    (half + rng.choice(len(gs) - half, args.batch_loop_sample // 2, replace=False)).tolist())
    for h in [int(x) for x in args.batch_hs.split(",")]:
        te = 0
        for G in Gs:
            te += kh.hdeg(G, h)[1]
        torch.cuda.synchronize()
        t = time.perf_counter()
        cores, res = kh.core_batch(Gs, h)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t
        log(f"batch h={h}: {tb:.2f}s")
        t = time.perf_counter()
        same = True
        te_s = 0
        for i in sample:
            c, _ = kh.core(Gs[i], h)
            same &= bool(np.array_equal(c, cores[i]))
        torch.cuda.synchronize()
        tl = time.perf_counter() - t
        for i in sample:
            te_s += kh.hdeg(Gs[i], h)[1]
        loop_est = tl * te / max(te_s, 1)
        out[f"h{h}"] = {"seconds": round(tb, 3), "graphs_per_s": round(len(gs) / tb, 2),
                        "edges_traversed_per_s": te / tb, "edges_traversed": te,
                        "rounds": res[0]["rounds"],
                        "loop_sample": {"graphs": len(sample), "seconds": round(tl, 3),
                                        "edges_traversed": te_s, "identical_to_batch": same},
                        "loop_estimate_s": round(loop_est, 2), "speedup_vs_loop": round(loop_est / tb, 2)}
    return out


def bench_serve(kh, ctx, args):
    """Serving workload: a pool of Chung-Lu graphs (gamma 2.2, average degree
    10, n lognormal with median 20000 and sigma 1.0 clipped to [1000, cap], one
    graph of exactly cap vertices); Poisson arrivals at --serve-qps for
    --serve-seconds, each request a uniform graph, h uniform in {2, 3} and mode
    uniform in {exact, eps = 0.5}.  Latency = arrival to result ready.  Requests
    still queued --serve-grace seconds after the last arrival are withdrawn and
    reported as unserved (latency percentiles cover the completed ones)."""
    import numpy as np
    import torch

    import graphgen as gg
    t0 = time.time()
    cap = args.serve_max_n
    sizes = gg.lognormal_sizes(args.serve_pool, 20_000, 1.0, 1_000, cap, 5)
    sizes[0] = cap
    gs = [gg.chung_lu(int(n), 5 * int(n), 2.2, seed=100 + i) for i, n in enumerate(sizes)]
    Gs = [kh.Graph.from_gg(ctx, g) for g in gs]
    torch.cuda.synchronize()
    log(f"serve pool: {len(gs)} graphs, {int(sizes.sum())} vertices, built in {time.time() - t0:.1f}s")
    rng = np.random.default_rng(11)
    nreq = int(args.serve_qps * args.serve_seconds)
    arrivals = np.cumsum(rng.exponential(1.0 / args.serve_qps, nreq))
    picks = rng.integers(len(gs), size=nreq)
    hs = rng.integers(2, 4, size=nreq)
    modes = rng.random(nreq) < 0.5
    srv = kh.Server(ctx, workers=args.serve_workers)
    t_start = time.perf_counter()
    done = {}
    pending = []
    i = 0
    last_log = 0.0
    cancelled = 0
    deadline = args.serve_seconds + args.serve_grace
    while i < nreq or pending:
        now = time.perf_counter() - t_start
        while i < nreq and arrivals[i] <= now:
            eps = 0.5 if modes[i] else 0.0
            kw = dict(seed=1, lazy_init=int(hs[i]) in args.lazy_set) if eps > 0 else {}
            tk = srv.submit(Gs[picks[i]], int(hs[i]), epsilon=eps, **kw)
            pending.append((tk, i))
            i += 1
        still = []
        for tk, j in pending:
            r = srv.poll(tk)
            if r is None:
                still.append((tk, j))
            else:
                done[j] = time.perf_counter() - t_start - arrivals[j]
        pending = still
        if now - last_log >= 5.0:
            log(f"serve t={now:.0f}s submitted {i} done {len(done)} pending {len(pending)}")
            last_log = now
        if now > deadline and i >= nreq:
            # withdraw what still waits in the queue; let the running ones finish
            rest = []
            for tk, j in pending:
                if srv.cancel(tk):
                    cancelled += 1
                else:
                    rest.append((tk, j))
            while rest:
                still = []
                for tk, j in rest:
                    if srv.poll(tk) is None:
                        still.append((tk, j))
                    else:
                        done[j] = time.perf_counter() - t_start - arrivals[j]
                rest = still
                now = time.perf_counter() - t_start
                if now - last_log >= 5.0:
                    log(f"serve t={now:.0f}s: waiting for {len(rest)} running requests, done {len(done)}")
                    last_log = now
                time.sleep(0.002)
            pending = []
        time.sleep(0.0005)
    wall = time.perf_counter() - t_start
    srv.stop()
    fin = sorted(done)
    lat = np.array([done[j] for j in fin])
    cls = {}
    for idx, j in enumerate(fin):
        key = f"{'sampled' if modes[j] else 'exact'}_h{int(hs[j])}"
        cls.setdefault(key, []).append(lat[idx])
    return {"requests": nreq, "completed": len(fin), "withdrawn_unserved": cancelled,
            "qps_offered": args.serve_qps, "seconds_offered": args.serve_seconds,
            "wall_s": round(wall, 3), "qps_served": round(len(fin) / wall, 2),
            "p50_ms": round(1e3 * percentile(lat, 50), 3) if lat.size else None,
            "p99_ms": round(1e3 * percentile(lat, 99), 3) if lat.size else None,
            "max_ms": round(1e3 * float(lat.max()), 3) if lat.size else None, "workers": args.serve_workers,
            "pool": {"graphs": len(gs), "max_n": int(cap), "median_n": int(np.median(sizes))},
            "per_class": {k: {"n": len(v), "p50_ms": round(1e3 * percentile(v, 50), 3),
                              "p99_ms": round(1e3 * percentile(v, 99), 3)} for k, v in sorted(cls.items())}}


def bench_cl4m(kh, ctx, args):
    """Large power-law workload (Chung-Lu n = 4,000,000, m = 60,000,000,
    gamma = 2.3): sampled Core at h = 3 for each epsilon in --cl4m-eps with the
    densest-core estimate (Alg. 7, pruning variant); then the deviation of the
    sampled core numbers from the exact ones on a smaller graph of the same
    family (n = --dev-n, average degree 30), where ExactCore is affordable."""
    import numpy as np
    import torch

    import graphgen as gg
    out = {}
    t0 = time.time()
    g = gg.workload("cl4m") if not args.dev_only else gg.empty(1)
    if not args.dev_only:
        log(f"cl4m generated in {time.time() - t0:.1f}s")
    G = kh.Graph.from_gg(ctx, g)
    core_out = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    for eps in ([] if args.dev_only else [float(x) for x in args.cl4m_eps.split(",")]):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, res = kh.core(G, 3, epsilon=eps, delta=0.05, seed=1, out=core_out, dense=not args.cl4m_no_dense,
                         prune=True, lazy_init=3 in args.lazy_set)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        log(f"cl4m sampled h=3 eps={eps}: {dt:.1f}s")
        out[f"eps{eps}"] = {"seconds": round(dt, 3), "with_alg7": not args.cl4m_no_dense, **{k: res[k] for k in (
            "M_used", "M_dense_used", "rounds", "max_core", "dense_k", "dense_size", "dense_density",
            "list_elements")}}
    del G
    # deviation from exact on a smaller graph of the same family
    n = args.dev_n
    gs = gg.chung_lu(n, 15 * n, 2.3, seed=2)
    Gs = kh.Graph.from_gg(ctx, gs)
    t = time.perf_counter()
    ex, rex = kh.core(Gs, 3)
    tex = time.perf_counter() - t
    log(f"deviation graph n={n}: exact h=3 {tex:.1f}s")
    dev = {"graph": f"chung_lu n={n} m={15 * n} gamma=2.3 seed=2", "h": 3, "exact_seconds": round(tex, 3),
           "exact_rounds": rex["rounds"], "exact_max_core": rex["max_core"]}
    exv = ex.astype(np.float64)
    for eps in [float(x) for x in args.cl4m_eps.split(",")]:
        t = time.perf_counter()
        sc, rs = kh.core(Gs, 3, epsilon=eps, delta=0.05, seed=1, lazy_init=3 in args.lazy_set)
        ts = time.perf_counter() - t
        pos = exv > 0
        ratio = sc[pos].astype(np.float64) / exv[pos]
        M = rs["M_used"]
        dev[f"eps{eps}"] = {
            "seconds": round(ts, 3), "M_used": M, "max_rel_dev": float(np.max(np.abs(ratio - 1.0))),
            "mean_rel_dev": float(np.mean(np.abs(ratio - 1.0))),
            "frac_within_eps": float(np.mean(np.abs(ratio - 1.0) <= eps)),
            "frac_exact": float(np.mean(sc == ex)),
            "frac_exact_where_core_lt_M": float(np.mean((sc == ex)[ex < M])) if np.any(ex < M) else None,
            "frac_core_lt_M": float(np.mean(ex < M))}
        log(f"deviation eps={eps}: {dev[f'eps{eps}']}")
    out["deviation"] = dev
    return out


def bench_sbm(kh, ctx, args):
    """The paper's scaling experiment (Sec. 8): hierarchical block models with
    10 equal blocks (inter-block pair probability 1e-6 i^2, intra-block 4e-4)
    at each n in --sbm-ns, sampled Core at eps = 0.5 and h = 2, 3, 4, with
    ExactCore beside it.  Each time is the median of --sbm-reps runs after one
    warm-up run, graph resident on the GPU, core numbers left on the device."""
    import torch

    import graphgen as gg
    rows = []
    for n in [int(x) for x in args.sbm_ns.split(",")]:
        g = gg.sbm(n, seed=1)
        G = kh.Graph.from_gg(ctx, g)
        out = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda:0")
        for h in (2, 3, 4):
            row = {"n": n, "m": g.m, "h": h}
            for mode, eps in (("sampled", 0.5), ("exact", 0.0)):
                ts = []
                for _ in range(args.sbm_reps + 1):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    _, res = kh.core(G, h, epsilon=eps, delta=0.05, seed=1, out=out)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t)
                row[f"{mode}_ms"] = round(1e3 * sorted(ts[1:])[len(ts[1:]) // 2], 3)
                row[f"{mode}_max_core"] = res["max_core"]
                row[f"{mode}_rounds"] = res["rounds"]
                if mode == "sampled":
                    row["M_used"] = res["M_used"]
            log(f"sbm {row}")
            rows.append(row)
        del G
    return {"graph": "sbm: 10 equal blocks, p(C_i,C_j)=1e-6 i^2 (i<j), p_in=4e-4, seed 1", "eps": 0.5,
            "rows": rows}


T_PROCESS_START = time.time()


def elapsed_total():
    return time.time() - T_PROCESS_START


def plan_counts(requested, est_step_s, left_s, minimum):
    """How many steps of est_step_s seconds fit into left_s (at least `minimum`,
    at most `requested`)."""
    if est_step_s <= 0:
        return requested
    return max(minimum, min(requested, int(left_s // est_step_s)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall-clock budget of the whole run; warmup and timed steps are cut to fit")
    ap.add_argument("--step-estimate-s", type=float, default=120.0,
                    help="assumed step time before one has been measured (decides whether a warmup step fits)")
    ap.add_argument("--stages", default="exact,sampled", help="comma list of hdeg,exact,sampled")
    ap.add_argument("--hs", default="2,3")
    ap.add_argument("--lazy-hs", default="3",
                    help="h values at which the sampled stage uses the lazy initialisation of the top level "
                         "(Sec. 5 heuristic; output-neutral); empty: none")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle work per h (all host cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--batch", action="store_true", help="also measure the batch workload (kh_core_batch)")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-hs", default="2,3")
    ap.add_argument("--batch-loop-sample", type=int, default=32)
    ap.add_argument("--serve", action="store_true", help="also measure the serving workload (kh_serve_*)")
    ap.add_argument("--serve-qps", type=float, default=200.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--serve-max-n", type=int, default=2_000_000)
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-grace", type=float, default=60.0,
                    help="seconds after the last arrival before queued requests are withdrawn")
    ap.add_argument("--cl4m", action="store_true", help="also measure the 4M-vertex sampled workload")
    ap.add_argument("--cl4m-eps", default="0.5,0.25")
    ap.add_argument("--cl4m-no-dense", action="store_true", help="--cl4m: Core only, without Alg. 7")
    ap.add_argument("--dev-n", type=int, default=100_000)
    ap.add_argument("--dev-only", action="store_true", help="--cl4m: only the deviation study")
    ap.add_argument("--sbm", action="store_true", help="also measure the block-model scaling series")
    ap.add_argument("--sbm-ns", default=",".join(str(10_000 * i) for i in range(1, 11)))
    ap.add_argument("--sbm-reps", type=int, default=3)
    ap.add_argument("--skip-main", action="store_true",
                    help="only the --batch / --serve / --cl4m / --sbm measurements")
    ap.add_argument("--trace-hops", default=None, metavar="KERNEL_TRACE_CSV",
                    help="summarise the exact peel's mask-BFS hops from a rocprofv3 kernel trace and exit")
    ap.add_argument("--pmc-out", default=None, help="--pmc-summarize: write here instead of profiles/")
    ap.add_argument("--no-prewarm", action="store_true",
                    help="skip the small-graph warm-up (counter runs: only the timed step's dispatches)")
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_counters.json from two rocprofv3 --pmc runs of this command")
    args = ap.parse_args()
    if args.trace_hops:
        trace_hops(args.trace_hops)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the build has no multi-GPU path, "
                                   "so --gpus must be 1"}))
        sys.exit(2)

    stages = [s for s in args.stages.split(",") if s]
    hs = [int(x) for x in args.hs.split(",")]
    lazy_hs = {int(x) for x in args.lazy_hs.split(",") if x}
    args.lazy_set = lazy_hs
    if args.pmc_summarize:
        pmc_summarize(args.pmc_summarize[0], args.pmc_summarize[1], stages, hs, args.pmc_out)
        return

    import concurrent.futures

    import graphgen as gg
    # the library's round loops print a line every 20 s of a long decomposition
    os.environ.setdefault("KH_HEARTBEAT", "20")
    # generate the benchmark graph while torch and the library load
    gen_pool = concurrent.futures.ThreadPoolExecutor(1)
    g_future = None if args.skip_main else gen_pool.submit(gg.workload, "cl1m")
    import torch

    import paper_2112_06154_amd as kh
    log(f"[{elapsed_total():.0f}s] torch and the library loaded")

    if args.skip_main:
        torch.cuda.set_device(0)
        ctx = kh.Context(0)
        extra = {}
        if args.batch:
            extra["batch"] = bench_batch(kh, ctx, args)
        if args.serve:
            extra["serve"] = bench_serve(kh, ctx, args)
        if args.cl4m:
            extra["cl4m"] = bench_cl4m(kh, ctx, args)
        if args.sbm:
            extra["sbm"] = bench_sbm(kh, ctx, args)
        print(json.dumps(extra))
        return

    torch.cuda.set_device(0)
    ctx = kh.Context(0)
    # load the kernels and run every stage once on a small graph of the same family
    small = gg.chung_lu(20_000, 200_000, 2.1, seed=3)
    Gs = kh.Graph.from_gg(ctx, small)
    outs = torch.empty(small.n, dtype=torch.int32, device="cuda:0")
    for h in ([] if args.no_prewarm else hs):
        kh.core(Gs, h, out=outs, dense=True, prune=True)
        kh.core(Gs, h, epsilon=0.5, delta=0.05, seed=1, out=outs, dense=True, prune=True, lazy_init=h in lazy_hs)
    torch.cuda.synchronize()
    del Gs
    g = g_future.result()
    gen_pool.shutdown()
    log(f"[{elapsed_total():.0f}s] graph {WORKLOAD} ready; small-graph prewarm done")
    G = kh.Graph.from_gg(ctx, g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()

    if args.copy_calib:
        # plain kernels of known traffic for the counter calibration: a fill
        # writing 1 GiB and an add reading 1 GiB and writing 1 GiB
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.add(a, 1, out=b)
        torch.cuda.synchronize()
        del a, b

    def step(record, tag):
        """One pass of the hot path; returns (exact TE, exact s, sampled list elements, sampled s)."""
        te = ex_s = le = sa_s = 0
        for h in hs:
            if "hdeg" in stages:
                t = time.perf_counter()
                _, te_h = kh.hdeg(G, h, out=out)
                torch.cuda.synchronize()
                record.setdefault(f"hdeg_h{h}_s", []).append(round(time.perf_counter() - t, 3))
                record[f"hdeg_h{h}_edges_traversed"] = te_h
            if "exact" in stages:
                t = time.perf_counter()
                _, res = kh.core(G, h, out=out, dense=True, prune=True)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                record.setdefault(f"exact_h{h}_s", []).append(round(dt, 3))
                record[f"exact_h{h}"] = {k: res[k] for k in ("rounds", "max_core", "dense_k", "dense_size",
                                                              "dense_density", "edges_traversed", "arcs_scanned")}
                te += res["edges_traversed"]
                ex_s += dt
                log(f"[{elapsed_total():.0f}s] {tag} exact h={h}: {dt:.2f}s, {res['rounds']} rounds")
            if "sampled" in stages:
                t = time.perf_counter()
                _, res = kh.core(G, h, epsilon=0.5, delta=0.05, seed=1, out=out, dense=True, prune=True,
                                 lazy_init=h in lazy_hs)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                record.setdefault(f"sampled_h{h}_s", []).append(round(dt, 3))
                record[f"sampled_h{h}"] = {k: res[k] for k in ("rounds", "max_core", "M_used", "M_dense_used",
                                                                "dense_k", "dense_size", "dense_density",
                                                                "list_elements")}
                le += res["list_elements"]
                sa_s += dt
                log(f"[{elapsed_total():.0f}s] {tag} sampled h={h}: {dt:.2f}s, {res['rounds']} rounds")
        return te, ex_s, le, sa_s

    # warmup: only while a warmup step and at least one timed step (plus the
    # CPU baseline) still fit into the budget
    reserve = 0.0 if args.no_cpu else args.cpu_budget * len(hs) + 5.0
    est = args.step_estimate_s
    warm = {}
    warm_done = 0
    for i in range(args.warmup):
        left = args.budget_s - elapsed_total() - reserve
        # timed steps come first: a warmup step beyond the first runs only if
        # every requested timed step still fits after it
        need = 2.0 * est if warm_done == 0 else est * 1.05 * (args.steps + 1)
        if left < need:
            log(f"[{elapsed_total():.0f}s] warmup cut at {warm_done} step(s): {left:.0f}s left, step ~{est:.0f}s")
            break
        t = time.perf_counter()
        step(warm, f"warmup {i + 1}")
        est = time.perf_counter() - t if warm_done == 0 else max(est, time.perf_counter() - t)
        warm_done += 1
    left = args.budget_s - elapsed_total() - reserve
    steps = plan_counts(args.steps, est * 1.05, left, 1)
    log(f"[{elapsed_total():.0f}s] timing {steps} step(s) of ~{est:.0f}s ({left:.0f}s left in the budget)")

    rec = {}
    ctx.profile(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    te_total = ex_total = le_total = sa_total = 0
    for i in range(steps):
        te, ex_s, le, sa_s = step(rec, f"step {i + 1}/{steps}")
        te_total += te
        ex_total += ex_s
        le_total += le
        sa_total += sa_s
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    profs = [ctx.profile_read(0), ctx.profile_read(1), ctx.profile_read(2)]
    ctx.profile(False)

    names = ["k_ms_pull (bit-parallel h-degree pull hop)", "k_union (sample-list union, levels >= 2)",
             "k_rbfs_hop (exact peel: one push or pull hop of the deleted set's mask BFS)"]

    def roofline(k):
        p = profs[k]
        ms = p["ms"]
        achieved = (p["alg_bytes"] / (ms * 1e-3)) / 1e9 if ms > 0 else 0.0
        r = {"kernel": names[k], "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
             "traffic": measured_traffic(k, stages, hs),
             "launches": p["launches"], "total_ms": round(ms, 2),
             "share_of_step": round(ms * 1e-3 / elapsed, 4) if elapsed > 0 else None,
             "avg_launch_ms": round(ms / max(p["launches"], 1), 4),
             "alg_bytes_per_launch": p["alg_bytes"] // max(p["launches"], 1)}
        if k == 0:
            r["gather_bytes_per_launch"] = p["gather_bytes"] // max(p["launches"], 1)
            r["gather_gbs"] = round((p["gather_bytes"] / (ms * 1e-3)) / 1e9, 2) if ms > 0 else 0.0
        return r

    order = sorted(range(len(profs)), key=lambda k: -profs[k]["ms"])
    dom = order[0]
    exact_rate = te_total / ex_total if ex_total > 0 else None
    line = {
        "metric": "(k,h)-core edges-traversed/sec + %HBM roofline at h=2,3",
        "value": exact_rate, "unit": "edges_traversed/s", "n_gpus": 1, "steps": steps,
        "warmup": warm_done, "ms_per_step": elapsed * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": WORKLOAD, "h": hs, "stages": stages, "epsilon": 0.5, "delta": 0.05,
                   "densest_core": "core levels, pruning variant", "lazy_init_at_h": sorted(lazy_hs),
                   "value": "ExactCore edges traversed (kh_result) / ExactCore wall time"},
        "requested": {"steps": args.steps, "warmup": args.warmup, "budget_s": args.budget_s},
        "exact": {"edges_traversed": te_total, "seconds": round(ex_total, 3),
                  "edges_traversed_per_s": exact_rate},
        "sampled": {"list_elements": le_total, "seconds": round(sa_total, 3),
                    "list_elements_per_s": le_total / sa_total if sa_total > 0 else None},
        "step_edges_traversed_per_s": te_total / elapsed if elapsed > 0 else None,
        "roofline": roofline(dom),
        "roofline_other": [roofline(k) for k in order[1:]],
        "stages_detail": rec,
    }
    if args.batch:
        line["batch"] = bench_batch(kh, ctx, args)
    if args.serve:
        line["serve"] = bench_serve(kh, ctx, args)
    if args.cl4m:
        line["cl4m"] = bench_cl4m(kh, ctx, args)
    if args.sbm:
        line["sbm"] = bench_sbm(kh, ctx, args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(g, hs, args.cpu_budget)
    line["wall_s_total"] = round(elapsed_total(), 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
