#!/usr/bin/env python3
"""Benchmark of the pull-PageRank path on one MI355X.

Workload (one "step"): the damping-factor sweep of the paper's section 2 -- eleven rank
vectors for alpha = 0.50, 0.55, ..., 1.00 -- on a seeded R-MAT graph of scale 24 (16,777,216
vertices, edge factor 16, a,b,c,d = .57,.19,.19,.05, seed 24, duplicates and self-loops removed),
each solved to tau = 1e-10 in the L-infinity norm (section 3) from the uniform start, max 500
iterations, all eleven together in one batched solve (pr_pull_batch; float32 gather with
float64 norms, teleport terms and final float64 updates).  The graph is synthetic: the paper's
SuiteSparse graphs are not available.

Reported:
  value          column-edge updates per second of the timed sweep (sum over the eleven columns
                 of E * iterations, divided by the step time), in GTEPS
  sweep          per-column iterations, the same sweep as eleven sequential float64 solves
                 (time and speed-up), errors against them, L1 distance to the alpha=0.85 ranks
  roofline       the dominant kernel's algorithmic bytes per launch over its average launch
                 duration, timed with HIP events on the solve stream inside the timed steps
  cpu_baseline   the CPU oracle (FP64, OpenMP gather) timed on a bounded sample of the same graph
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "α-sweep time to τ=1e-10 vs plain FP64; GTEPS; HBM GB/s as % of peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench %7.1fs]" % (time.time() - T0), *a, file=sys.stderr, flush=True)


T0 = time.time()


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag, digest):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None when the summary is
    missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", kernel_tag + "_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        m = re.match(r"^([a-z_0-9]+):\s*(\S+)", line.strip())
        if m:
            kv[m.group(1)] = m.group(2)
    if kv.get("source_digest") != digest:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--seed", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--calibrate", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--path", choices=["batch_mixed", "batch_fp64"], default="batch_mixed",
                    help="the timed sweep: batched mixed precision (default) or batched float64")
    ap.add_argument("--seq-reps", type=int, default=2, help="timed repetitions of the sequential FP64 sweep")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    import paper_2108_02997_amd as pr

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)

    log("generating R-MAT scale %d seed %d" % (args.scale, args.seed))
    g = gg.rmat(args.scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=args.seed)
    N, E = g.N, g.E
    log("graph N=%d E=%d dangling=%d" % (N, E, int((g.outdeg == 0).sum())))
    ctx = pr.Context(0)
    dg = pr.DeviceGraph.from_host(g, 0)
    t = time.time()
    dg.prepare(ctx)
    torch.cuda.synchronize()
    prep_ms = (time.time() - t) * 1e3
    log("prepared in %.1f ms" % prep_ms)

    alphas = gg.ALPHA_SWEEP
    tau, norm, max_iter = 1e-10, pr.PR_LINF, 500
    problems = [dict(alpha=a, tau=tau, norm=norm, max_iter=max_iter) for a in alphas]
    K = len(problems)
    ranks_b = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in alphas]
    ranks_s = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in alphas]
    batch_prec = pr.PR_FP64 if args.path == "batch_fp64" else pr.PR_MIXED

    def sweep_batch():
        return pr.pull_batch(ctx, dg, problems, precision=batch_prec, ranks=ranks_b)

    def sweep_sequential():
        return [pr.pull(ctx, dg, alpha=p["alpha"], tau=tau, norm=norm, max_iter=max_iter, precision=pr.PR_FP64,
                        ranks=r) for p, r in zip(problems, ranks_s)]

    if args.calibrate:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        copy_gbs = 10 * 2 * src.numel() * 4 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
        log("device copy 1 GiB: %.0f GB/s (read+write)" % copy_gbs)
        del src, dst

    def timed(fn, reps, tag):
        ts, out = [], None
        for i in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            log("%s %d: %.2f ms" % (tag, i + 1, ts[-1] * 1e3))
        return ts, out

    # the plain FP64 reference: 11 sequential solves (untimed warm-up, then timed)
    sweep_sequential()
    seq_times, seq_res = timed(sweep_sequential, args.seq_reps, "sequential fp64 sweep")
    seq_s = float(np.mean(seq_times))

    for i in range(args.warmup):
        sweep_batch()
        log("warmup %d done" % (i + 1))
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    times, results = timed(sweep_batch, args.steps, "step (batched sweep)")
    ctx.set_option("timing", 0)
    step_s = float(np.mean(times))
    iters = [r["iterations"] for r in results]
    col_edges = sum(E * k for k in iters)
    gteps = col_edges / step_s / 1e9

    # dominant kernel: the batched update of the first phase (float32 for the mixed path).
    # Algorithmic bytes of one launch with K_a active columns: 4E (indices) + 4(N+1) (offsets)
    # + 4N (out-degrees) + 2*s*K_a*N (read and write of the active columns, s bytes each).
    dom_kind = pr._lib.PR_KERNEL_BATCH_F32 if batch_prec == pr.PR_MIXED else pr._lib.PR_KERNEL_BATCH_F64
    s_bytes = 4 if batch_prec == pr.PR_MIXED else 8
    phase1 = [r["fp32_iters"] for r in results] if batch_prec == pr.PR_MIXED else iters
    n_dom, ms_dom = ctx.stats(dom_kind)
    launches = max(phase1)
    alg = [4 * E + 4 * (N + 1) + 4 * N + 2 * s_bytes * N * sum(1 for k in phase1 if k > i) for i in range(launches)]
    alg_per_launch = float(np.mean(alg))
    avg_launch_s = (ms_dom / n_dom) * 1e-3 if n_dom else float("nan")
    achieved = alg_per_launch / avg_launch_s / 1e9
    n_f64, ms_f64 = ctx.stats(pr._lib.PR_KERNEL_BATCH_F64)
    kname = "k_batch_update<float,%d>" % (4 if K > 8 else (K + 3) // 4) if batch_prec == pr.PR_MIXED else \
        "k_batch_update<double,%d>" % ((K + 3) // 4)
    digest = source_digest(["paper_2108_02997_amd/csrc/batch.hip", "paper_2108_02997_amd/csrc/batch.h",
                            "paper_2108_02997_amd/csrc/internal.h"])
    traffic = read_traffic("batch_update_%s_rmat_s%d" % ("f32" if s_bytes == 4 else "f64", args.scale), digest)

    # section 2 report: L1 distance of every column to the alpha = 0.85 column; and the batched
    # result against the sequential FP64 solves
    i85 = list(alphas).index(0.85)
    l1_vs_085 = [pr.l1_distance(ctx, r["ranks"], results[i85]["ranks"]) for r in results]
    l1_vs_fp64 = [pr.l1_distance(ctx, rb, rs) for rb, rs in zip(ranks_b, ranks_s)]
    linf_vs_fp64 = [float((rb - rs).abs().max()) for rb, rs in zip(ranks_b, ranks_s)]

    line = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if batch_prec == pr.PR_MIXED else "f64",
        "data": "synthetic",
        "config": {
            "workload": "alpha sweep: 11 rank columns alpha=0.50..1.00 solved together to tau=1e-10 (Linf) on R-MAT "
                        "scale %d, edge factor 16, (.57,.19,.19,.05), seed %d; %s" % (
                            args.scale, args.seed, "float32 gather + float64 norms/c0/refinement"
                            if batch_prec == pr.PR_MIXED else "float64"),
            "N": N, "E": E, "tau": tau, "norm": "Linf", "max_iter": max_iter, "path": args.path,
        },
        "roofline": {
            "kernel": kname,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": round(alg_per_launch),
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
            "launches_timed": n_dom,
        },
        "sweep": {
            "alphas": list(alphas), "iterations": iters, "fp32_iters": [r["fp32_iters"] for r in results],
            "fp64_iters": [r["fp64_iters"] for r in results], "converged": [r["converged"] for r in results],
            "column_edges": col_edges, "prep_ms": round(prep_ms, 2),
            "sequential_fp64_ms": round(seq_s * 1e3, 3),
            "sequential_fp64_iterations": [r["iterations"] for r in seq_res],
            "speedup_vs_sequential_fp64": round(seq_s / step_s, 3),
            "l1_vs_alpha_085": [round(x, 6) for x in l1_vs_085],
            "l1_vs_sequential_fp64": l1_vs_fp64, "linf_vs_sequential_fp64": linf_vs_fp64,
            "batch_f64_update_us": round(1e3 * ms_f64 / n_f64, 2) if n_f64 else None,
        },
    }

    if not args.no_cpu:
        import oracle
        log("cpu oracle sample")
        t = time.perf_counter()
        oracle.pagerank_graph(g, alpha=0.85, tau=0.0, norm=oracle.L1, max_iter=1)
        t1 = time.perf_counter() - t
        k = int(max(1, min(40, round(args.cpu_seconds / max(t1, 1e-3)))))
        t = time.perf_counter()
        oracle.pagerank_graph(g, alpha=0.85, tau=0.0, norm=oracle.L1, max_iter=k)
        tk = time.perf_counter() - t
        line["cpu_baseline"] = {
            "value": round(E * k / tk / 1e9, 4), "unit": "GTEPS", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d FP64 oracle iterations (alpha=0.85) over the full graph, %.1f s; host CPU %s"
                      % (k, tk, cpu_model()),
        }
        log("cpu oracle: %d iterations in %.2f s" % (k, tk))
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
