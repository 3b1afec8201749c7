"""Benchmark: exact kNN queries/s on one MI355X through libkdtree's C ABI.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload uniform-1m] [--k 8]

One step = one kd_knn call over the whole query batch (query reorder +
stack-free traversal + results in caller order), inputs already resident in
HBM, outputs preallocated.  The tree is built once, untimed.  Prints ONE JSON
line.  The roofline figure is for the traversal kernel: algorithmic bytes =
processed nodes x dim x 4 B (node data touched), divided by the kernel's mean
duration from hipEvents recorded around each launch on its own stream.

The headline ("plain") is the paper's traversal: the far child is pruned by
its split plane only (kd_opts.prune = 1).  The same line carries the
library's default rule, which also leaves a subtree on entry when its
bounding box is out of range ("boxes", identical results, fewer nodes), the
learned-radius variant on the same queries ("learned", paper's rule), a
batched many-tree measurement ("batched") and the CPU oracle timed on the
host ("cpu_baseline"); each can be skipped by a flag.

Other measurements, each printing its own JSON line instead of the headline:
  --paper-grid   the shape of the paper's Table 1 (4-D, N 1K..200M, 10M queries)
  --range        radius and box search on the 1M-point 3-D workloads
  --split-rules  level-rule trees against stored widest-extent dimensions
  --copy-calibration  a plain 1 GiB copy, the reference for HBM counters
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "kNN queries/sec (k=8, 1M pts) plain vs learned-radius; % HBM peak"
HBM_PEAK_GBPS = 8000.0
PLAIN = {"prune": 1}  # the paper's split-plane pruning rule

WORKLOADS = {
    "uniform-1m": "N=1,048,576 uniform float32 3-D points in [0,1)^3 (seed 0); Q=1,048,576 uniform queries (seed 1)",
    "gmm64-1m": "N=1,048,576 float32 3-D points from a 64-cluster Gaussian mixture (sigma 0.01); Q=1,048,576 from the same mixture",
    "uniform-16k": "N=16,384 uniform float32 3-D points; Q=16,384 uniform queries",
    "clustered-10m": "N=10,000,000 float32 3-D points, 256-cluster mixture (sigma log-uniform 0.002-0.05); Q=10,000,000 (90% mixture, 10% uniform)",
    "shells-100m": "N=100,000,000 float32 3-D points on 1000 sphere shells (radius 0.01-0.1, radial noise 1e-4); Q=100,000,000 near the shells",
    "uniform4d-1m-q10m": "N=1,048,576 uniform float32 4-D points in [0,1)^4 (seed 0); Q=10,000,000 uniform queries (seed 1): the shape of the paper's Table 1",
}
DEFAULT_RADIUS = {"shells-100m": 0.005}  # else unbounded


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def src_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_counters(kernel_key: str, cur_hash: str):
    """The committed rocprofv3 --pmc summary of the kernel, if it was taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != cur_hash:
        return None
    return d


def load_traffic(kernel_key: str, cur_hash: str, launches_units: float):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source; else None."""
    d = load_counters(kernel_key, cur_hash)
    return None if d is None else d.get("hbm_bytes_per_launch")


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(P, Qs, k, reps=3, single_sample=1 << 18):
    """The oracle (plain recursive traversal, C, one thread per host core
    with dynamic chunks) on the workload's queries, best of reps; plus the
    same on one thread over the first single_sample queries."""
    import oracle
    order = oracle.build_tree(P)  # untimed
    threads = oracle.default_threads()

    def best_of(qs, nthreads):
        best = math.inf
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.knn(P, order, qs, k, nthreads=nthreads)
            best = min(best, time.perf_counter() - t0)
        return qs.shape[0] / best

    value = best_of(Qs, threads)
    one = best_of(Qs[:single_sample], 1)
    return dict(value=value, unit="queries/s", cores=threads, kind="oracle",
                sample=f"all {Qs.shape[0]} queries of the workload, k={k}, recursive traversal, "
                       f"best of {reps}, tree built untimed",
                value_1_core=one, sample_1_core=f"first {min(single_sample, Qs.shape[0])} queries, 1 thread, "
                                                f"best of {reps}",
                cpu_model=host_cpu_model(), host_threads=os.cpu_count())


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain copy kernel of known size: each launch reads and writes nbytes.
    rocprofv3 FETCH_SIZE / WRITE_SIZE of this kernel give the counters' scale."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "launches": reps}), flush=True)


def bench_boxes(kd, tree, q, oi, od, k, args, plain_ms):
    """The library's default pruning rule on the same queries (kd_knn with no
    options): split planes plus subtree bounding boxes.  Timed like the plain
    step; results checked identical to the plain results."""
    import torch
    dev = q.device
    bi = torch.empty_like(oi)
    bd = torch.empty_like(od)
    kd.kd_knn(tree, q, k, args.max_radius, out_idx=bi, out_d2=bd)
    _, _, vis = kd.kd_knn_ex(tree, q, k, args.max_radius, want_visited=True, opts={"prune": 2})
    torch.cuda.synchronize()
    identical = bool(torch.equal(bi, oi) and torch.equal(bd.view(torch.int32), od.view(torch.int32)))
    entered = int(vis.to(torch.int64).sum().item())
    for _ in range(args.warmup):
        kd.kd_knn(tree, q, k, args.max_radius, out_idx=bi, out_d2=bd)
    torch.cuda.synchronize()
    kd.kd_timing_enable(True)
    kd.kd_timing_collect("traverse")
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        kd.kd_knn(tree, q, k, args.max_radius, out_idx=bi, out_d2=bd)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    tot, n = kd.kd_timing_collect("traverse")
    kd.kd_timing_enable(False)
    value = q.shape[0] / (ms / 1e3)
    log(f"boxes: {ms:.3f} ms/step, {value / 1e6:.1f} M queries/s ({plain_ms / ms:.3f}x plain), "
        f"entered {entered / q.shape[0]:.1f}/query, identical {identical}")
    return {"value": value, "unit": "queries/s", "ms_per_step": ms, "traverse_ms": tot / max(1, n),
            "speedup_vs_plain": plain_ms / ms, "identical_to_plain": identical,
            "entered_per_query": entered / q.shape[0]}


def bench_learned(kd, datagen, tree, q, oi, od, k, args, plain_visited, plain_ms):
    """Learned initial radius on the same queries: train (untimed) on separate
    queries of the same distribution, then time kd_knn_learned like the plain
    step.  Results are checked identical to the plain results."""
    import torch
    dev = q.device
    train = torch.from_numpy(datagen.training_queries(args.workload, 1 << 20, 7)).to(dev)
    t0 = time.perf_counter()
    model = kd.kd_radius_model_train(tree, train, k, epochs=args.train_epochs, batch=8192, seed=0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    info = model.info()
    log(f"learned: trained in {train_s:.2f}s, holdout rmse {info['holdout_rmse']:.3f}, margin {info['margin']:.3f}")
    li = torch.empty_like(oi)
    ld = torch.empty_like(od)
    vis = torch.empty(q.shape[0], dtype=torch.int32, device=dev)
    _, _, _, st = kd.kd_knn_learned(tree, model, q, k, args.max_radius, out_idx=li, out_d2=ld, visited=vis,
                                    want_stats=True, opts=PLAIN)
    torch.cuda.synchronize()
    identical = bool(torch.equal(li, oi) and torch.equal(ld.view(torch.int32), od.view(torch.int32)))
    lvis = int(vis.to(torch.int64).sum().item())
    for _ in range(args.warmup):
        kd.kd_knn_learned(tree, model, q, k, args.max_radius, out_idx=li, out_d2=ld, opts=PLAIN)
    torch.cuda.synchronize()
    kd.kd_timing_enable(True)
    for name in ("sort", "mlp", "traverse", "fallback"):
        kd.kd_timing_collect(name)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        kd.kd_knn_learned(tree, model, q, k, args.max_radius, out_idx=li, out_d2=ld, opts=PLAIN)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    stages = {}
    for name in ("sort", "mlp", "traverse", "fallback"):
        tot, n = kd.kd_timing_collect(name)
        stages[name + "_ms"] = tot / max(1, n)
    kd.kd_timing_enable(False)
    model.close()
    value = q.shape[0] / (ms / 1e3)
    log(f"learned: {ms:.3f} ms/step, {value / 1e6:.1f} M queries/s ({plain_ms / ms:.3f}x plain), "
        f"fallbacks {st['fallbacks']}, identical {identical}")
    return {"value": value, "unit": "queries/s", "ms_per_step": ms, "speedup_vs_plain": plain_ms / ms,
            "identical_to_plain": identical, "fallbacks": st["fallbacks"], "visited_per_query": lvis / q.shape[0],
            "visited_ratio_vs_plain": lvis / plain_visited, "train_s": train_s, "train_queries": int(train.shape[0]),
            "epochs": args.train_epochs, "holdout_rmse": info["holdout_rmse"], "margin": info["margin"], **stages}


def bench_batched(kd, datagen, args):
    """Many trees in one captured launch pipeline: the batched workload (512
    trees, N log-uniform [1K, 2M], D in {2,3,4}, uniform or GMM-64, k in
    {1,8,32}, Q = N), trees built untimed.  Timed: kd_batch_run (hipGraph
    replay of the whole pipeline) per step with the default options, then
    after the batch autotuner (untimed) picked options per (dim, k) group,
    against the same jobs as one kd_knn call each.  Results are checked
    identical.  Roofline: node bytes of the entered nodes (the default rule's
    count, summed over the jobs) per replay of the whole pipeline."""
    import torch
    dev = torch.device("cuda:0")
    jobs_meta = datagen.batched_jobs(args.batch_jobs, seed=42, n_max=args.batch_nmax)
    jobs, single = [], []
    t0 = time.perf_counter()
    for m in jobs_meta:
        P, Qs = datagen.job_arrays(m)
        tree = kd.kd_build(torch.from_numpy(P).to(dev))
        q = torch.from_numpy(Qs).to(dev)
        Q, k = q.shape[0], m["k"]
        jobs.append(dict(tree=tree, queries=q, k=k, out_idx=torch.empty((Q, k), dtype=torch.int32, device=dev),
                         out_d2=torch.empty((Q, k), dtype=torch.float32, device=dev)))
        single.append((torch.empty((Q, k), dtype=torch.int32, device=dev),
                       torch.empty((Q, k), dtype=torch.float32, device=dev)))
    torch.cuda.synchronize()
    log(f"batched: {len(jobs)} trees built in {time.perf_counter() - t0:.1f}s (untimed)")
    total_q = sum(j["queries"].shape[0] for j in jobs)
    # entered nodes under the default rule (the batch's), node bytes summed
    alg_bytes = 0
    for j in jobs:
        _, _, v = kd.kd_knn_ex(j["tree"], j["queries"], j["k"], want_d2=False, want_visited=True,
                               opts={"prune": 2})
        alg_bytes += int(v.to(torch.int64).sum().item()) * j["queries"].shape[1] * 4
    batch = kd.Batch(jobs)
    stream = torch.cuda.current_stream()

    def run_single():
        for j, (oi, od) in zip(jobs, single):
            kd.kd_knn(j["tree"], j["queries"], j["k"], out_idx=oi, out_d2=od)

    def timed(fn, steps):
        for _ in range(max(5, args.warmup)):  # first replays of a fresh graph run slower
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_d = timed(lambda: batch.run(stream), args.steps)
    t0 = time.perf_counter()
    tuned = batch.autotune(reps=2, stream=stream)
    tune_s = time.perf_counter() - t0
    ms_b = timed(lambda: batch.run(stream), args.steps)
    ms_s = timed(run_single, max(1, args.steps // 4))
    identical = all(torch.equal(j["out_idx"], oi) and torch.equal(j["out_d2"].view(torch.int32), od.view(torch.int32))
                    for j, (oi, od) in zip(jobs, single))
    groups = batch.info()
    batch.close()
    learned = None
    if args.batch_learned:
        # the same batch with a radius model per 3-D job of at least 2^16
        # points (trained untimed on queries of the job's own distribution,
        # another seed), default plans, against the plain default-plan replay
        t0 = time.perf_counter()
        models = []
        for m, j in zip(jobs_meta, jobs):
            if m["dim"] != 3 or m["n"] < (1 << 16):
                continue
            _, tq = datagen.job_arrays(dict(m, query_seed=m["query_seed"] + 10007))
            model = kd.kd_radius_model_train(j["tree"], torch.from_numpy(tq).to(dev), j["k"], epochs=4,
                                             batch=8192, seed=0)
            j["model"] = model
            models.append(model)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        lbatch = kd.Batch(jobs)
        ms_l = timed(lambda: lbatch.run(stream), args.steps)
        same = all(torch.equal(j["out_idx"], oi) and torch.equal(j["out_d2"].view(torch.int32), od.view(torch.int32))
                   for j, (oi, od) in zip(jobs, single))
        lbatch.close()
        for j in jobs:
            j.pop("model", None)
        for model in models:
            model.close()
        learned = {"ms_per_step": ms_l, "value": total_q / (ms_l / 1e3), "unit": "queries/s",
                   "speedup_vs_plain_default_options": ms_d / ms_l, "models": len(models),
                   "train_s": train_s, "identical_to_single_calls": same}
        log(f"batched learned: {ms_l:.3f} ms/step ({ms_d / ms_l:.3f}x the plain replay), {len(models)} models, "
            f"identical {same}")
    for j in jobs:
        j["tree"].close()
    achieved = alg_bytes / (ms_b / 1e3) / 1e9
    log(f"batched: default {ms_d:.3f} ms/step, tuned {ms_b:.3f} ms/step ({total_q / ms_b / 1e3:.1f} M queries/s), "
        f"one call per tree {ms_s:.3f} ms/step, identical {identical}")
    return {"value": total_q / (ms_b / 1e3), "unit": "queries/s", "ms_per_step": ms_b, "jobs": len(jobs),
            "total_queries": total_q, "ms_per_step_default_options": ms_d, "autotune_s": tune_s,
            "tuned_options": [dict(dim=g[0], K=g[1], queries=g[2], **o) for g, o in zip(groups, tuned)],
            "ms_per_step_one_call_per_tree": ms_s, "speedup_vs_one_call_per_tree": ms_s / ms_b,
            "identical_to_single_calls": identical,
            "learned": learned,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBPS, "alg_bytes_per_replay": alg_bytes,
                         "timed": "whole graph replay (sort, gather, traversal, hand-off of every group)"},
            "sample": f"{len(jobs)} trees, N log-uniform [1000, {args.batch_nmax}], D in {{2,3,4}}, uniform or "
                      f"GMM-64, k in {{1,8,32}}, Q = N, seed 42; hipGraph replay per step"}


# The paper's Table 1 (RTX 3090 Ti, uniform float4 points in [0,1]^4, 10M
# uniform queries; queries/s).  Context only: another GPU, another generation.
PAPER_TABLE1 = {
    1_000: [888e6, 563e6, 359e6, 48e6, 14e6, 5.2e9, 6.6e9, 4.0e9, 1.8e9],
    10_000: [664e6, 407e6, 262e6, 29.5e6, 8.7e6, 3.3e9, 3.9e9, 3.3e9, 1.6e9],
    100_000: [396e6, 184e6, 122e6, 20.6e6, 6.0e6, 1.7e9, 1.8e9, 1.7e9, 1.1e9],
    1_000_000: [100e6, 42.1e6, 26.6e6, 7.5e6, 2.9e6, 334e6, 338e6, 282e6, 255e6],
    10_000_000: [44e6, 19.3e6, 12.3e6, 5.0e6, 2.3e6, 58.2e6, 58.5e6, 52.8e6, 51e6],
    100_000_000: [36e6, 16.5e6, 10.8e6, 4.7e6, 2.1e6, 19.1e6, 16.6e6, 14.2e6, 13.8e6],
    200_000_000: [34.8e6, 16.2e6, 10.6e6, 4.5e6, 2.1e6, 16.7e6, 12.2e6, 9.2e6, 8.9e6],
}
PAPER_COLUMNS = [(1, math.inf), (4, math.inf), (8, math.inf), (20, math.inf), (50, math.inf),
                 (4, 0.01), (8, 0.01), (20, 0.01), (50, 0.01)]  # (k, maxRadius); k = 1 is fcp


def paper_grid(args):
    """The shape of the paper's Table 1 on this GPU: 4-D uniform points in
    [0,1)^4, N from 1K to 200M, 10M uniform queries, fcp and kNN k in
    {4, 8, 20, 50} unbounded and within 0.01; queries/s of one call (query
    reorder + traversal), under the paper's pruning rule and the library
    default, each checked on sampled rows against the oracle's brute force."""
    import numpy as np
    import torch

    import oracle
    import paper_2210_12859_amd as kd
    from paper_2210_12859_amd import datagen
    dev = torch.device("cuda:0")
    Qs = datagen.uniform(10_000_000, 4, 1)
    q = torch.from_numpy(Qs).to(dev)
    stream = torch.cuda.current_stream()
    rows_out = []
    for N in sorted(PAPER_TABLE1):
        P = datagen.uniform(N, 4, 0)
        tree = kd.kd_build(torch.from_numpy(P).to(dev))
        nrows = 32 if N <= 10_000_000 else 4
        rows = np.random.default_rng(N).choice(len(Qs), nrows, replace=False)
        for col, (k, maxr) in enumerate(PAPER_COLUMNS):
            oi = torch.empty((len(Qs), k), dtype=torch.int32, device=dev)
            od = torch.empty((len(Qs), k), dtype=torch.float32, device=dev)
            cell = {"N": N, "k": k, "maxRadius": maxr, "paper_qps": PAPER_TABLE1[N][col]}
            bi, bd = oracle.brute(P, Qs[rows], k, maxr)
            for name, opts in (("paper_rule", {"prune": 1}), ("default", None)):
                kd.kd_knn_ex(tree, q, k, maxr, out_idx=oi, out_d2=od, opts=opts)
                torch.cuda.synchronize()
                r = torch.from_numpy(rows).to(dev)
                ok = bool(np.array_equal(oi[r].cpu().numpy(), bi) and
                          np.array_equal(od[r].cpu().numpy().view(np.uint32), bd.view(np.uint32)))
                reps = 3
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    kd.kd_knn_ex(tree, q, k, maxr, out_idx=oi, out_d2=od, opts=opts)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                cell[name + "_qps"] = len(Qs) / (ms / 1e3)
                cell[name + "_exact_on_sample"] = ok
            log(f"paper grid N={N} k={k} maxR={maxr:g}: {cell['paper_rule_qps'] / 1e6:.1f} M q/s (paper rule), "
                f"{cell['default_qps'] / 1e6:.1f} M q/s (default), paper {cell['paper_qps'] / 1e6:.1f} M q/s")
            rows_out.append(cell)
            del oi, od
        tree.close()
        del P
    print(json.dumps({"paper_grid": rows_out, "queries": len(Qs),
                      "workload": "uniform float32 4-D points in [0,1)^4 (seed 0); 10,000,000 uniform queries (seed 1)",
                      "note": "paper_qps: the paper's Table 1, RTX 3090 Ti; context only"}), flush=True)


def range_queries(args):
    """Radius and box search (the un-ordered traversal) on the 1M-point 3-D
    workloads: regions sized for a mean of 8 and 64 points on uniform data,
    results kept for the 8 nearest / smallest indices or counts only.  Per
    cell and pruning mode (split planes only, the paper's traversal and the
    default; subtree bounding boxes on request): queries/s of one call (Morton
    reorder + traversal), the traversal kernel's average duration from the
    library's events on the call's stream, entered nodes per query; for split
    planes also the HBM roofline fraction of the entered nodes' coordinates;
    and exactness of 256 sampled rows against the oracle's definitions."""
    import numpy as np
    import torch

    import oracle
    import paper_2210_12859_amd as kd
    from paper_2210_12859_amd import datagen
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cells = []
    for wl in ("uniform-1m", "gmm64-1m"):
        P, Qs = datagen.workload(wl)
        N, D = P.shape
        Q = Qs.shape[0]
        tree = kd.kd_build(torch.from_numpy(P).to(dev))
        q = torch.from_numpy(Qs).to(dev)
        rows = np.random.default_rng(0).choice(Q, 256, replace=False)
        r_t = torch.from_numpy(rows).to(dev)
        vis = torch.empty(Q, dtype=torch.int32, device=dev)
        for kind, m, cap in (("radius", 8, 8), ("radius", 64, 0), ("box", 8, 8), ("box", 64, 0)):
            if kind == "radius":
                size = (3.0 * m / (4.0 * math.pi * N)) ** (1.0 / 3.0)
                oc, oi, od = oracle.radius(P, Qs[rows], size, cap)
            else:
                size = 0.5 * (m / N) ** (1.0 / 3.0)  # half-width of a cube holding m points on average
                lo_np = Qs - np.float32(size)
                hi_np = Qs + np.float32(size)
                lo = torch.from_numpy(lo_np).to(dev)
                hi = torch.from_numpy(hi_np).to(dev)
                oc, oi = oracle.box(P, lo_np[rows], hi_np[rows], cap)
            cell = {"workload": wl, "kind": kind, "size": size, "cap": cap}
            for mode, flags in (("planes", 0), ("boxes", kd.KD_RANGE_BOXES)):
                if kind == "radius":
                    call = lambda v=None, f=flags: kd.kd_radius_search(tree, q, size, cap, visited=v, flags=f)
                else:
                    call = lambda v=None, f=flags: kd.kd_box_search(tree, lo, hi, cap, visited=v, flags=f)
                res = call(vis)
                torch.cuda.synchronize()
                entered = int(vis.to(torch.int64).sum().item())
                cnt = res[0][r_t].cpu().numpy().astype(np.int64)
                ok = bool(np.array_equal(cnt, oc))
                if cap:
                    ok = ok and bool(np.array_equal(res[1][r_t].cpu().numpy(), oi))
                    if kind == "radius":
                        ok = ok and bool(np.array_equal(res[2][r_t].cpu().numpy().view(np.uint32), od.view(np.uint32)))
                cell["mean_count"] = float(res[0].to(torch.float64).mean().item())
                for _ in range(args.warmup):
                    call()
                torch.cuda.synchronize()
                kd.kd_timing_enable(True)
                kd.kd_timing_collect(kind)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(args.steps):
                    call()
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                kt, kn = kd.kd_timing_collect(kind)
                kd.kd_timing_enable(False)
                kern_ms = kt / max(1, kn)
                cell[mode] = {"qps": Q / (ms / 1e3), "ms_per_call": ms, "kernel_ms": kern_ms,
                              "entered_per_query": entered / Q, "exact_on_sample": ok}
                if mode == "planes":
                    alg = entered * D * 4
                    cell[mode]["alg_bytes_per_launch"] = alg
                    cell[mode]["roofline_frac"] = alg / (kern_ms / 1e3) / 1e9 / HBM_PEAK_GBPS
            # the oracle (the plain definition, brute force over all N points,
            # one thread per host core) on a bounded sample of the same queries
            ns = 2048
            t0 = time.perf_counter()
            if kind == "radius":
                oracle.radius(P, Qs[:ns], size, cap)
            else:
                oracle.box(P, lo_np[:ns], hi_np[:ns], cap)
            cell["cpu_baseline"] = {"value": ns / (time.perf_counter() - t0), "unit": "queries/s",
                                    "cores": oracle.default_threads(), "kind": "oracle",
                                    "sample": f"first {ns} queries, brute force over all {N} points"}
            pl, df = cell["planes"], cell["boxes"]
            log(f"{wl} {kind} size={size:.4g} cap={cap}: {cell['mean_count']:.1f} in range; planes "
                f"{pl['qps'] / 1e6:.1f} M q/s, kernel {pl['kernel_ms']:.3f} ms, entered {pl['entered_per_query']:.1f}, "
                f"frac {pl['roofline_frac']:.3f}; boxes {df['qps'] / 1e6:.1f} M q/s, kernel {df['kernel_ms']:.3f} ms, "
                f"entered {df['entered_per_query']:.1f} ({pl['kernel_ms'] / df['kernel_ms']:.2f}x); "
                f"oracle {cell['cpu_baseline']['value'] / 1e3:.1f} K q/s; "
                f"exact {pl['exact_on_sample'] and df['exact_on_sample']}")
            cells.append(cell)
        # every point in range (offsets + indices): counting pass, scan, fill
        import ctypes
        L = kd.lib()
        st = ctypes.c_void_p(stream.cuda_stream)
        # (uniform data only: the same region sizes hold ~10^4 clustered
        # points each, 10^10 results over 1M queries)
        for kind, m in ((("radius", 64), ("box", 64)) if wl == "uniform-1m" else ()):
            if kind == "radius":
                size = (3.0 * m / (4.0 * math.pi * N)) ** (1.0 / 3.0)
                src = q
            else:
                size = 0.5 * (m / N) ** (1.0 / 3.0)
                src = torch.stack([torch.from_numpy(Qs - np.float32(size)), torch.from_numpy(Qs + np.float32(size))],
                                  dim=1).contiguous().to(dev)
            off = torch.empty(Q + 1, dtype=torch.int64, device=dev)
            tot = ctypes.c_int64()

            def run_all(out, cap):
                if kind == "radius":
                    rc = L.kd_radius_search_all(tree.handle, ctypes.c_void_p(src.data_ptr()), Q, size,
                                                ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(out), cap,
                                                ctypes.byref(tot), 0, st)
                else:
                    rc = L.kd_box_search_all(tree.handle, ctypes.c_void_p(src.data_ptr()), Q,
                                             ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(out), cap,
                                             ctypes.byref(tot), 0, st)
                assert rc == 0, L.kd_last_error().decode()

            run_all(None, 0)
            out = torch.empty(max(1, tot.value), dtype=torch.int32, device=dev)
            for _ in range(max(1, args.warmup)):
                run_all(out.data_ptr(), tot.value)
            t0 = time.perf_counter()
            reps = max(1, args.steps // 2)
            for _ in range(reps):
                run_all(out.data_ptr(), tot.value)
            ms = (time.perf_counter() - t0) * 1e3 / reps  # the call synchronises
            cell = {"workload": wl, "kind": kind + "_all", "size": size, "total_results": tot.value,
                    "qps": Q / (ms / 1e3), "results_per_s": tot.value / (ms / 1e3), "ms_per_call": ms}
            log(f"{wl} {kind} all results size={size:.4g}: {tot.value} results, {ms:.3f} ms/call, "
                f"{cell['qps'] / 1e6:.1f} M q/s, {cell['results_per_s'] / 1e9:.2f} G results/s")
            cells.append(cell)
            del out, off, src
        tree.close()
    print(json.dumps({"range_queries": cells, "steps": args.steps, "warmup": args.warmup,
                      "note": "radius: ball of radius size; box: cube of half-width size around each query"}),
          flush=True)


def split_rules(args):
    """Trees whose split dimension is the level's against trees that store
    each node's widest extent, on the same points and queries: build time
    (untimed elsewhere), processed nodes per query under the paper's rule,
    and the traversal time of one call under the paper's rule and under the
    library default (subtree boxes).  Both trees give the same exact rows,
    which is checked on every query."""
    import numpy as np
    import torch

    import paper_2210_12859_amd as kd
    from paper_2210_12859_amd import datagen
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cells = []
    for wl, k in (("uniform-1m", 8), ("gmm64-1m", 8), ("clustered-10m", 16), ("shells-100m", 32)):
        maxr = DEFAULT_RADIUS.get(wl, math.inf)
        P, Qs = datagen.workload(wl)
        p = torch.from_numpy(P).to(dev)
        q = torch.from_numpy(Qs).to(dev)
        del P, Qs
        Q = q.shape[0]
        res = {}
        for name, split in (("level", kd.KD_SPLIT_LEVEL), ("widest", kd.KD_SPLIT_WIDEST)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tree = kd.kd_build(p, split=split)
            build_s = time.perf_counter() - t0
            oi = torch.empty((Q, k), dtype=torch.int32, device=dev)
            od = torch.empty((Q, k), dtype=torch.float32, device=dev)
            vis = torch.empty(Q, dtype=torch.int32, device=dev)
            kd.kd_knn_ex(tree, q, k, maxr, out_idx=oi, out_d2=od, visited=vis)
            torch.cuda.synchronize()
            cell = {"build_s": build_s, "visited_per_query": float(vis.to(torch.float64).mean().item())}
            del vis
            for rule, opts in (("paper_rule", PLAIN), ("default", None)):
                kd.kd_knn_ex(tree, q, k, maxr, out_idx=oi, out_d2=od, opts=opts)
                reps = 3 if Q <= 10_000_000 else 1
                kd.kd_timing_enable(True)
                kd.kd_timing_collect("traverse")
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    kd.kd_knn_ex(tree, q, k, maxr, out_idx=oi, out_d2=od, opts=opts)
                e1.record(stream)
                torch.cuda.synchronize()
                kt, kn = kd.kd_timing_collect("traverse")
                kd.kd_timing_enable(False)
                cell[rule + "_ms"] = e0.elapsed_time(e1) / reps
                cell[rule + "_traverse_ms"] = kt / max(1, kn)
            res[name] = (cell, oi, od)
            tree.close()
        if wl != "shells-100m":
            # the oracle over the widest tree (recursive traversal with stored
            # dimensions, one thread per host core) on a bounded sample
            import oracle
            Pn = p.cpu().numpy()
            qn = q[: 1 << 16].cpu().numpy()
            order, dims = oracle.build_tree_widest(Pn)  # untimed
            t0 = time.perf_counter()
            oracle.knn(Pn, order, qn, k, maxr, dims=dims)
            res["widest"][0]["cpu_baseline"] = {
                "value": qn.shape[0] / (time.perf_counter() - t0), "unit": "queries/s",
                "cores": oracle.default_threads(), "kind": "oracle",
                "sample": f"first {qn.shape[0]} queries, recursive traversal over the widest tree"}
            del Pn, qn, order, dims
        li, ld = res["level"][1], res["level"][2]
        wi, wd = res["widest"][1], res["widest"][2]
        same = bool(torch.equal(li, wi) and torch.equal(ld.view(torch.int32), wd.view(torch.int32)))
        row = {"workload": wl, "k": k, "maxRadius": maxr, "identical_rows": same,
               "level": res["level"][0], "widest": res["widest"][0]}
        lv, wv = row["level"], row["widest"]
        log(f"{wl} k={k}: visited {lv['visited_per_query']:.1f} -> {wv['visited_per_query']:.1f}, paper rule "
            f"{lv['paper_rule_ms']:.2f} -> {wv['paper_rule_ms']:.2f} ms, default {lv['default_ms']:.2f} -> "
            f"{wv['default_ms']:.2f} ms, build {lv['build_s']:.3f} -> {wv['build_s']:.3f} s, identical {same}")
        cells.append(row)
        del res, li, ld, wi, wd, p, q
        torch.cuda.empty_cache()
    print(json.dumps({"split_rules": cells}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform-1m", choices=sorted(WORKLOADS))
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--max-radius", type=float, default=None,
                    help="search radius (default: 0.005 for shells-100m, else unbounded)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-radius variant")
    ap.add_argument("--no-boxes", action="store_true", help="skip the default (bounding-box) pruning variant")
    ap.add_argument("--train-epochs", type=int, default=8)
    ap.add_argument("--batch-jobs", type=int, default=512, help="trees in the batched measurement (0 = skip)")
    ap.add_argument("--batch-nmax", type=int, default=2000000, help="largest tree of the batched measurement")
    ap.add_argument("--batch-learned", action="store_true",
                    help="also time the batch with a radius model per large 3-D job")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--paper-grid", action="store_true",
                    help="only run the shape of the paper's Table 1 (4-D, N 1K..200M, 10M queries)")
    ap.add_argument("--split-rules", action="store_true",
                    help="only compare level-rule trees with stored widest-extent dimensions")
    ap.add_argument("--range", action="store_true",
                    help="only run the radius and box search measurement (1M-point 3-D workloads)")
    args = ap.parse_args()
    if args.range:
        range_queries(args)
        return
    if args.split_rules:
        split_rules(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.paper_grid:
        paper_grid(args)
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(queries shard trivially across GPUs with a replicated tree; "
                                   "see the design notes)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2210_12859_amd as kd
    from paper_2210_12859_amd import datagen

    if args.max_radius is None:
        args.max_radius = DEFAULT_RADIUS.get(args.workload, math.inf)
    dev = torch.device("cuda:0")
    k = args.k
    log(f"workload {args.workload} k={k}: generating inputs")
    P, Qs = datagen.workload(args.workload)
    N, D = P.shape
    Q = Qs.shape[0]
    t0 = time.perf_counter()
    tree = kd.kd_build(torch.from_numpy(P).to(dev))
    log(f"tree built in {time.perf_counter() - t0:.2f}s (untimed)")
    q = torch.from_numpy(Qs).to(dev)
    oi = torch.empty((Q, k), dtype=torch.int32, device=dev)
    od = torch.empty((Q, k), dtype=torch.float32, device=dev)
    vis = torch.empty(Q, dtype=torch.int32, device=dev)

    # processed nodes per query (deterministic; equals the oracle's count)
    kd.kd_knn_ex(tree, q, k, args.max_radius, out_idx=oi, out_d2=od, visited=vis)
    torch.cuda.synchronize()
    visited_total = int(vis.to(torch.int64).sum().item())
    log(f"mean processed nodes/query = {visited_total / Q:.2f}")

    for _ in range(args.warmup):
        kd.kd_knn_ex(tree, q, k, args.max_radius, out_idx=oi, out_d2=od, opts=PLAIN)
    torch.cuda.synchronize()
    kd.kd_timing_enable(True)
    kd.kd_timing_collect("traverse")
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        kd.kd_knn_ex(tree, q, k, args.max_radius, out_idx=oi, out_d2=od, opts=PLAIN)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    kern_ms, launches = kd.kd_timing_collect("traverse")
    kd.kd_timing_enable(False)
    ms_per_step = total_ms / args.steps
    kern_avg_ms = kern_ms / max(1, launches)
    value = Q / (ms_per_step / 1e3)
    log(f"{ms_per_step:.3f} ms/step, traversal kernel {kern_avg_ms:.3f} ms, {value / 1e6:.1f} M queries/s")

    alg_bytes = visited_total * D * 4  # node data touched per launch
    achieved = alg_bytes / (kern_avg_ms / 1e3) / 1e9
    cur_hash = src_hash(["paper_2210_12859_amd/csrc/kd_traverse.hip", "paper_2210_12859_amd/csrc/kd_internal.h"])
    traffic = load_traffic(f"traverse_{args.workload}_k{k}", cur_hash, 1)
    counters = load_counters(f"traverse_{args.workload}_k{k}", cur_hash)
    # the secondary algorithmic total: node data plus each query read and its
    # k results (index + squared distance) written by the same kernel
    alg2 = alg_bytes + Q * (D * 4 + k * 8)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}; kNN k={k}, maxRadius={args.max_radius:g}",
                   "variant": "plain", "k": k, "N": N, "Q": Q, "dim": D},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "knn_persistent (stack-free traversal)",
                     "kernel_ms": kern_avg_ms, "alg_bytes_per_launch": alg_bytes,
                     "secondary": {"alg_bytes_per_launch": alg2,
                                   "frac": alg2 / (kern_avg_ms / 1e3) / 1e9 / HBM_PEAK_GBPS,
                                   "note": "node data + query reads + result writes"},
                     "l2_hit_pct": counters.get("l2_hit_pct") if counters else None,
                     "valu_issue_pct": (100.0 * counters["sq_insts_valu"] * 4 /
                                        (1024 * kern_avg_ms * 1e-3 * 2.4e9)) if counters else None,
                     "source_hash": cur_hash},
        "visited_per_query": visited_total / Q,
        "nodes_visited_per_s": visited_total / (ms_per_step / 1e3),
    }
    if not args.no_boxes:
        out["boxes"] = bench_boxes(kd, tree, q, oi, od, k, args, ms_per_step)
    if not args.no_learned and D == 3:
        out["learned"] = bench_learned(kd, datagen, tree, q, oi, od, k, args, visited_total, ms_per_step)
    if args.batch_jobs > 0:
        out["batched"] = bench_batched(kd, datagen, args)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(P, Qs, k)
    print(json.dumps(out), flush=True)
    tree.close()


if __name__ == "__main__":
    main()
