#!/usr/bin/env python3
"""Benchmark of the pull-PageRank path on one MI355X.

Default workload (--workload sweep; one "step"): the damping-factor sweep of the paper's
section 2 -- eleven rank vectors for alpha = 0.50, 0.55, ..., 1.00 -- on a seeded R-MAT graph of
scale 24 (16,777,216 vertices, edge factor 16, a,b,c,d = .57,.19,.19,.05, seed 24, duplicates
and self-loops removed), each solved to tau = 1e-10 in the L-infinity norm (section 3) from the
uniform start, max 500 iterations, all eleven together.  Default path (--path series): one
float64 iteration serves all eleven columns (pr_pull_sweep: from the uniform start the iterate of
damping factor a is a^k v_k + (1-a) sum_{j<k} a^j v_j with v_j the a = 1 iterates, and its
change a^k times theirs), each column stopping exactly where its own iteration would; the batched
mixed-precision sweep (pr_pull_batch: float32 gather with float64 norms, teleport terms and final
float64 updates) is timed beside it (--path batch_mixed makes it the headline).  The graph is
synthetic: the paper's SuiteSparse graphs are not available; it is prepared with the
source-segmented layout (--seg-len, default 2^19 ids per segment).

Reported:
  value            column-edge updates per second of the timed sweep (sum over the eleven columns
                   of E * iterations, divided by the step time), in GTEPS
  batch_mixed      the batched mixed-precision sweep of the same columns (time, iterations, the
                   roofline of its dominant kernel), when the series path is the headline
  sweep            per-column iterations, the same sweep as eleven sequential float64 solves
                   (time and speed-up), errors against them, L1 distance to the alpha=0.85 ranks
  roofline         the dominant kernel's algorithmic bytes per launch over its average launch
                   duration, timed with HIP events on the solve stream in a pass of the same step
                   run right after the timed steps (the timed steps replay captured HIP graphs,
                   whose kernels events cannot bracket one by one);
                   beside it (after the timed steps) the bare gather of the same rows over the
                   same index array (microbench/gather_ceiling.hip), and the kernel's time as a
                   fraction of that bare time
  plain_fp64_gather  the same for the single-vector float64 update of the sequential solves
  warm_sweep       the same sweep with learned warm starts, the alpha=0.85 solve, features, inference
                   and the judge inside the timed step (and a variant without the judge)
  degree_order     the same sweep and sequential solves on the graph relabelled by out-degree
                   (pr_relabel, excluded from the timing like the prep), ranks mapped back
  cpu_baseline     the CPU oracle (FP64, OpenMP gather) timed on a bounded sample of the same graph:
                   the columns alpha = 0.85, 0.95, 1.00 solved in full, each compared with the
                   headline's column (iterations, L1, L-infinity)

Other workloads (one JSON line each, same keys):
  --workload small      Erdos-Renyi N=10,000 (average out-degree 8, 5% dangling), one float64 solve
                        to tau=1e-6 (L1): solve and update times, oracle on one and on all cores
  --workload tau        R-MAT scale 22: every (tau, norm) stop for tau = 1e-3 .. 1e-10 and the
                        three norms, float64 against mixed precision (iterations, time, distance),
                        with a float32-only ablation beside them (continued to 1e-12), the
                        sensitivity-issue and single-iteration checks of sections 4-5, and the
                        update times on the graph as generated, randomly relabelled (locality
                        stress case) and in out-degree order
  --workload multi      64 seeded graphs of uneven size (log-uniform 1e3 .. 1e6 vertices) with
                        their own alpha/tau/norm, autotuned, in one persistent launch, against
                        the sum of 64 sequential solves
  --workload norms      sections 3 and 4 on the same 64 graphs at alpha = 0.85: iterations and
                        times of L1/L2/Linf at tau = 1e-6 with the six composite ratios (tables
                        3.1/3.2), the 21-tolerance sweep read off one traced launch, and the same
                        readout on a 2048 x 2048 road-like lattice (single-iteration stops)
  --workload warmstart  the learned warm start: a network trained on 20 R-MAT scale-20 graphs
                        proposes start vectors for alpha = 0.90/0.95/0.99 on three unseen scale-24
                        graphs; iterations and time from the uniform, alpha=0.85 and learned starts;
                        roofline of the float64 update, and of the network's inference on the
                        matrix cores (float32 MFMA peak)
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
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense float32 matrix-core peak of the MI355X
CSRC = "paper_2108_02997_amd/csrc/"


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


def timed(fn, reps, tag):
    import torch
    ts, out = [], None
    for i in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        log("%s %d: %.2f ms" % (tag, i + 1, ts[-1] * 1e3))
    return ts, out


def single_update_bytes(N, E, s):
    """Algorithmic bytes of one single-vector update: indices, offsets, out-degrees, read and
    write of the s-byte state."""
    return 4 * E + 4 * (N + 1) + 4 * N + 2 * s * N


def roofline(kernel, alg_bytes, avg_s, launches, traffic):
    achieved = alg_bytes / avg_s / 1e9
    out = {"kernel": kernel, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "algorithmic_bytes_per_launch": round(alg_bytes), "avg_launch_us": round(avg_s * 1e6, 2),
           "launches_timed": launches}
    if traffic:
        # the measured HBM-side bytes (calibrated counters) over the same launch time
        out["traffic_GBps"] = round(traffic / avg_s / 1e9, 1)
        out["traffic_frac_of_peak"] = round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4)
    return out


def bare_gather_us(dg, row_bytes):
    """Time of the bare gather of one `row_bytes` row per in-edge of `dg` (index stream plus row
    fetches, nothing else; microbench/gather_ceiling.hip), in us; None when not measurable."""
    try:
        from paper_2108_02997_amd.microbench import gather_ceiling as gc
        if row_bytes not in gc.ROW_KINDS:
            return None
        return 1e3 * gc.bare_gather_ms(gc.load(), dg.idx, dg.N, row_bytes)
    except OSError as e:  # measurement library not built
        log("bare gather not measured: %s" % e)
        return None


def add_ceiling(entry, dg, row_bytes):
    """The kernel's launch time against the bare gather of its rows on the same graph."""
    bare = bare_gather_us(dg, row_bytes)
    if bare is not None:
        entry["bare_gather_us"] = round(bare, 1)
        entry["frac_of_bare_gather"] = round(bare / entry["avg_launch_us"], 4)


def stream_gbps(torch):
    """Achievable streaming bandwidth: a 1 GiB device-to-device copy (read + write bytes / time)."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline(graphs, seconds, what):
    """The oracle (FP64, OpenMP gather) timed on a bounded number of updates over `graphs`."""
    import oracle
    log("cpu oracle sample")
    t = time.perf_counter()
    for g in graphs:
        oracle.pagerank_graph(g, alpha=0.85, tau=0.0, norm=oracle.L1, max_iter=1)
    t1 = time.perf_counter() - t
    k = int(max(1, min(200, round(seconds / max(t1, 1e-3)))))
    t = time.perf_counter()
    for g in graphs:
        oracle.pagerank_graph(g, alpha=0.85, tau=0.0, norm=oracle.L1, max_iter=k)
    tk = time.perf_counter() - t
    edges = sum(g.E for g in graphs) * k
    log("cpu oracle: %d iterations in %.2f s" % (k, tk))
    return {"value": round(edges / tk / 1e9, 4), "unit": "GTEPS", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d FP64 oracle iterations (alpha=0.85) over %s, %.1f s; host CPU %s" % (k, what, tk, cpu_model())}


def base_line(metric, value, unit, args, ms, dtype, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 3), "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic", "config": config}


# ------------------------------------------------------------------ the damping-factor sweep

def batch_roofline(pr, ctx, results, stat_steps, fp32, N, E, scale, dg, copy_gbs):
    """Roofline of the dominant kernel of a batched sweep: the first phase's update on the widest
    rows (the launches before the first compaction of the active columns).  Algorithmic bytes of
    one launch with K_a active columns: 4E (indices) + 4(N+1) (offsets) + 4N (out-degrees) +
    2*s*K_a*N (read and write of the active columns, s bytes each)."""
    s_bytes = 4 if fp32 else 8
    kp0 = max(w for w in pr._lib.BATCH_ROW_WIDTHS if ctx.stats(pr._lib.batch_kind(fp32, w))[0] > 0)
    phase1 = [r["fp32_iters"] for r in results] if fp32 else [r["iterations"] for r in results]
    n_dom, ms_dom = ctx.stats(pr._lib.batch_kind(fp32, kp0))
    per_step = max(1, round(n_dom / stat_steps))
    alg = [4 * E + 4 * (N + 1) + 4 * N + 2 * s_bytes * N * sum(1 for k in phase1 if k > i) for i in range(per_step)]
    avg_launch_s = (ms_dom / n_dom) * 1e-3 if n_dom else float("nan")
    digest = source_digest([CSRC + "batch.hip", CSRC + "batch.h", CSRC + "internal.h"])
    traffic = read_traffic("batch_update_%s_rmat_s%d" % ("f32" if fp32 else "f64", scale), digest)
    out = roofline("k_batch_update<%s,%d>" % ("float" if fp32 else "double", kp0), float(np_mean(alg)), avg_launch_s,
                   n_dom, traffic)
    out["frac_of_stream"] = round(out["achieved"] / copy_gbs, 4)
    add_ceiling(out, dg, kp0 * s_bytes)
    return out


def np_mean(x):
    return sum(x) / len(x)


def run_sweep(args, pr, gg, np, torch):
    scale = args.scale or 24
    seed = args.seed if args.seed is not None else 24
    log("generating R-MAT scale %d seed %d" % (scale, seed))
    g = gg.rmat(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=seed)
    N, E = g.N, g.E
    log("graph N=%d E=%d dangling=%d" % (N, E, int((g.outdeg == 0).sum())))
    ctx = pr.Context(0)
    dg = pr.DeviceGraph.from_host(g, 0)
    t = time.time()
    if args.seg_len:
        # tile partitions plus the source-segmented layout: single-vector updates (the sequential
        # float64 solves, the power-series sweep) run as per-segment partial sums and a merge
        dg.prepare_segmented(ctx, seg_len=args.seg_len)
    else:
        dg.prepare(ctx)
    torch.cuda.synchronize()
    prep_ms = (time.time() - t) * 1e3
    log("prepared in %.1f ms (segments of %d ids, %d pairs)" % (prep_ms, args.seg_len, dg.seg_pairs))

    alphas = gg.ALPHA_SWEEP
    tau, norm, max_iter = 1e-10, pr.PR_LINF, 500
    problems = [dict(alpha=a, tau=tau, norm=norm, max_iter=max_iter) for a in alphas]
    ranks_h = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in alphas]
    ranks_s = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in alphas]

    def sweep_series():
        return pr.pull_sweep(ctx, dg, problems, ranks=ranks_h)

    def sweep_batch(prec, ranks):
        return pr.pull_batch(ctx, dg, problems, precision=prec, ranks=ranks)

    headline = {"series": sweep_series,
                "batch_mixed": lambda: sweep_batch(pr.PR_MIXED, ranks_h),
                "batch_fp64": lambda: sweep_batch(pr.PR_FP64, ranks_h)}[args.path]

    def sweep_sequential():
        return [pr.pull(ctx, dg, alpha=p["alpha"], tau=tau, norm=norm, max_iter=max_iter, precision=pr.PR_FP64,
                        ranks=r) for p, r in zip(problems, ranks_s)]

    # achievable streaming bandwidth (also the copy kernel that calibrates the memory counters)
    copy_gbs = stream_gbps(torch)
    log("device copy 1 GiB: %.0f GB/s (read+write)" % copy_gbs)

    # the plain FP64 reference: 11 sequential solves.  The first (untimed) pass runs with per-launch
    # event timing to measure the single-vector float64 update; the timed passes replay graphs.
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    sweep_sequential()
    ctx.set_option("timing", 0)
    n64, ms64 = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F64)
    # the same float64 update without the segmented layout (one solve, event-timed), for comparison
    plain64_us = None
    if args.seg_len:
        ctx.set_option("segmented", 0)
        ctx.reset_stats()
        ctx.set_option("timing", 1)
        pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm, max_iter=max_iter, precision=pr.PR_FP64)
        ctx.set_option("timing", 0)
        ctx.set_option("segmented", 1)
        a, b = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F64)
        plain64_us = 1e3 * b / a if a else None
    seq_times, seq_res = timed(sweep_sequential, args.seq_reps, "sequential fp64 sweep")
    seq_s = float(np.mean(seq_times))

    for i in range(args.warmup):
        headline()
        log("warmup %d done" % (i + 1))
    # the timed steps run as a caller runs them (captured update chunks replayed as HIP graphs)
    times, results = timed(headline, args.steps, "step (%s sweep)" % args.path)
    step_s = float(np.mean(times))
    # per-launch kernel times: HIP events cannot bracket the kernels of a replayed graph, so the
    # same step runs again with every update launched directly between two events on the solve
    # stream (option "timing"), right after the timed steps
    stat_steps = max(1, min(args.steps, 5))
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    ev_times, _ = timed(headline, stat_steps, "step with per-launch events")
    ctx.set_option("timing", 0)
    iters = [r["iterations"] for r in results]
    col_edges = sum(E * k for k in iters)
    gteps = col_edges / step_s / 1e9
    d64 = source_digest([CSRC + "pull.hip", CSRC + "device.h", CSRC + "internal.h", CSRC + "segment.hip"])
    traffic64 = read_traffic("update_f64_rmat_s%d" % scale, d64)
    b64 = single_update_bytes(N, E, 8)
    name64 = ("segmented float64 update (k_seg_gather<double> + k_update<double> merge + k_finish<double>)"
              if args.seg_len else "k_update<double>")

    extra = {}
    if args.path == "series":
        # dominant kernel: the a = 1 iteration's float64 update (one per update of the slowest column)
        nu, msu = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F64)
        nf, msf = ctx.stats(pr._lib.PR_KERNEL_SWEEP_FOLD)
        roof = roofline(name64, b64, msu / nu * 1e-3, nu, traffic64)
        roof["frac_of_stream"] = round(roof["achieved"] / copy_gbs, 4)
        add_ceiling(roof, dg, 8)
        # value counts every column's edge updates; the iteration itself gathers E edges per update
        # of the slowest column (its edge rate beside: gathered_edges_gteps)
        extra = {"updates_per_step": round(nu / stat_steps, 2), "update_us": round(1e3 * msu / nu, 1),
                 "folds_per_step": round(nf / stat_steps, 2), "fold_us": round(1e3 * msf / nf, 1) if nf else None,
                 "gathered_edges_gteps": round(nu / stat_steps * E / step_s / 1e9, 2)}
        dtype = "f64"
        how = ("float64, one iteration for all columns (PageRank as a power series in the damping factor: the a = 1 "
               "iterates v_j, column a's change a^k (v_k - v_{k-1}), ranks a^k v_k + (1-a) sum_{j<k} a^j v_j)")
    else:
        fp32 = args.path == "batch_mixed"
        roof = batch_roofline(pr, ctx, results, stat_steps, fp32, N, E, scale, dg, copy_gbs)
        dtype = "f32+f64" if fp32 else "f64"
        how = "float32 gather + float64 norms/c0/refinement" if fp32 else "float64 batch"

    # section 2 report: L1 distance of every column to the alpha = 0.85 column; and the sweep's
    # result against the sequential FP64 solves
    i85 = list(alphas).index(0.85)
    l1_vs_085 = [pr.l1_distance(ctx, r["ranks"], results[i85]["ranks"]) for r in results]
    l1_vs_fp64 = [pr.l1_distance(ctx, rb, rs) for rb, rs in zip(ranks_h, ranks_s)]
    linf_vs_fp64 = [float((rb - rs).abs().max()) for rb, rs in zip(ranks_h, ranks_s)]

    line = base_line(METRIC, round(gteps, 3), "GTEPS", args, step_s * 1e3, dtype, {
        "workload": "alpha sweep: 11 rank columns alpha=0.50..1.00 solved together to tau=1e-10 (Linf) on R-MAT "
                    "scale %d, edge factor 16, (.57,.19,.19,.05), seed %d; %s" % (scale, seed, how),
        "N": N, "E": E, "tau": tau, "norm": "Linf", "max_iter": max_iter, "path": args.path})
    line["roofline"] = roof
    if n64:
        line["plain_fp64_gather"] = roofline(name64, b64, ms64 / n64 * 1e-3, n64, traffic64)
        line["plain_fp64_gather"]["gteps_per_update"] = round(E / (ms64 / n64 * 1e-3) / 1e9, 2)
        line["plain_fp64_gather"]["frac_of_stream"] = round(line["plain_fp64_gather"]["achieved"] / copy_gbs, 4)
        if args.seg_len:
            line["plain_fp64_gather"]["segment_len"] = args.seg_len
            line["plain_fp64_gather"]["pairs"] = dg.seg_pairs
            line["plain_fp64_gather"]["unsegmented_update_us"] = round(plain64_us, 1) if plain64_us else None
            if plain64_us:
                line["plain_fp64_gather"]["unsegmented_frac"] = round(b64 / (plain64_us * 1e-6) / 1e9 /
                                                                      HBM_PEAK_GBS, 4)
        add_ceiling(line["plain_fp64_gather"], dg, 8)
    line["stream_copy_GBps"] = round(copy_gbs, 1)
    line["sweep"] = {
        "alphas": list(alphas), "iterations": iters, "fp32_iters": [r["fp32_iters"] for r in results],
        "fp64_iters": [r["fp64_iters"] for r in results], "converged": [r["converged"] for r in results],
        "column_edges": col_edges, "prep_ms": round(prep_ms, 2),
        "sequential_fp64_ms": round(seq_s * 1e3, 3),
        "sequential_fp64_iterations": [r["iterations"] for r in seq_res],
        "speedup_vs_sequential_fp64": round(seq_s / step_s, 3),
        "l1_vs_alpha_085": [round(x, 6) for x in l1_vs_085],
        "l1_vs_sequential_fp64": l1_vs_fp64, "linf_vs_sequential_fp64": linf_vs_fp64,
        "step_ms_min_median": [round(min(times) * 1e3, 3), round(float(np.median(times)) * 1e3, 3)],
        "step_ms_with_launch_events": round(float(np.mean(ev_times)) * 1e3, 3),
    }
    line["sweep"].update(extra)
    if args.path == "series":
        # the batched mixed-precision sweep of the same columns, timed beside it
        ranks_m = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in alphas]
        mixed = lambda: sweep_batch(pr.PR_MIXED, ranks_m)  # noqa: E731
        mixed()
        ts_m, res_m = timed(mixed, max(1, min(args.steps, 5)), "step (batched mixed sweep)")
        ctx.reset_stats()
        ctx.set_option("timing", 1)
        timed(mixed, 2, "batched mixed sweep with per-launch events")
        ctx.set_option("timing", 0)
        step_m = float(np.mean(ts_m))
        line["batch_mixed"] = {
            "step_ms": round(step_m * 1e3, 3), "gteps": round(sum(E * r["iterations"] for r in res_m) / step_m / 1e9, 3),
            "iterations": [r["iterations"] for r in res_m], "fp32_iters": [r["fp32_iters"] for r in res_m],
            "speedup_vs_sequential_fp64": round(seq_s / step_m, 3),
            "linf_vs_headline": [float((a - b).abs().max()) for a, b in zip(ranks_m, ranks_h)],
            "roofline": batch_roofline(pr, ctx, res_m, 2, True, N, E, scale, dg, copy_gbs)}
        del ranks_m
    if not args.no_warm:
        line["warm_sweep"] = warm_sweep(args, pr, gg, ctx, dg, problems, tau, norm, max_iter, step_s, iters, np, torch)
    if not args.no_relabel:
        line["degree_order"] = relabelled_sweep(args, pr, ctx, dg, problems, args.path, tau, norm, max_iter, N, E,
                                                step_s, seq_s, ranks_h, torch, np)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_sweep(g, problems, results, np)
    ctx.close()
    return line


def cpu_baseline_sweep(g, problems, results, np):
    """The oracle (FP64, OpenMP gather) timed on a bounded sample of the sweep: the columns alpha =
    0.85, 0.95 and 1.00 solved in full (tau = 1e-10, Linf, uniform start), each compared with the
    headline's column (iterations, L1 and L-infinity distance)."""
    import oracle
    log("cpu oracle sample: three full columns")
    pick = [i for i, p in enumerate(problems) if round(p["alpha"], 2) in (0.85, 0.95, 1.0)]
    spent, edges, cmp = 0.0, 0, {}
    for i in pick:
        p = problems[i]
        t = time.perf_counter()
        ref = oracle.pagerank_graph(g, alpha=p["alpha"], tau=p["tau"], norm=p["norm"], max_iter=p["max_iter"])
        spent += time.perf_counter() - t
        edges += g.E * ref["iterations"]
        d = np.abs(results[i]["ranks"].cpu().numpy() - ref["ranks"])
        cmp["%.2f" % p["alpha"]] = {"oracle_iterations": ref["iterations"], "gpu_iterations": results[i]["iterations"],
                                    "l1": float(d.sum()), "linf": float(d.max())}
    log("cpu oracle: %d edge visits in %.2f s" % (edges, spent))
    return {"value": round(edges / spent / 1e9, 4), "unit": "GTEPS", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "the columns alpha = 0.85, 0.95, 1.00 of the sweep solved in full by the FP64 oracle "
                      "(%d updates in all over the full graph, %.1f s); host CPU %s"
                      % (edges // g.E, spent, cpu_model()),
            "headline_vs_oracle": cmp}


def warm_sweep(args, pr, gg, ctx, dg, problems, tau, norm, max_iter, step_s, iters_uniform, np, torch):
    """The same sweep with learned warm starts (not part of the headline): the alpha = 0.85 column is
    solved first (mixed precision, uniform start); for every other alpha the network proposes a start
    from it (features + inference); the judge runs the candidate starts {network, alpha = 0.85 ranks,
    uniform} for three float64 updates as columns of one batch and keeps the smallest last change;
    then the ten remaining columns are solved together (mixed) from the judged iterates.  The timed
    step includes all of it.  A second variant skips the judge (network starts as proposed).  The
    network is trained first on ranks the method produces (R-MAT scale-20 graphs, seeds from 2000)."""
    from paper_2108_02997_amd import warmstart as wsm
    model = wsm.WarmStart(ctx, seed=0)
    train_alphas = [0.5, 0.55, 0.6, 0.65, 0.7, 0.75, 0.8, 0.85, 0.9, 0.95, 0.99]
    t0 = time.time()
    samples = []
    for s in range(args.warm_graphs):
        h = gg.rmat(20, edge_factor=16, seed=2000 + s)
        samples += model.make_samples(pr.DeviceGraph.from_host(h, 0), train_alphas)
    hist = model.train(samples, epochs=args.epochs, lr=3e-3)
    del samples
    torch.cuda.synchronize()
    train_s = time.time() - t0
    log("warm start: trained on %d graphs in %.1f s (loss %.4f -> %.4f)" % (args.warm_graphs, train_s, hist[0],
                                                                           hist[-1]))
    alphas = [p["alpha"] for p in problems]
    i85 = alphas.index(0.85)
    others = [p for i, p in enumerate(problems) if i != i85]

    def step(judged):
        r85 = pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm, max_iter=max_iter, precision=pr.PR_MIXED)
        starts, choices, look = [], [], 0
        for p in others:
            if judged:
                r0, name, _, steps, _ = model.start(dg, r85["ranks"], p["alpha"], norm=norm)
                look = steps
            else:
                r0, name = model.propose(dg, r85["ranks"], p["alpha"]), "mlp"
            starts.append(r0)
            choices.append(name)
        res = pr.pull_batch(ctx, dg, others, precision=pr.PR_MIXED, inits=starts)
        return r85, res, choices, look

    out = {"train_graphs": args.warm_graphs, "train_s": round(train_s, 2), "epochs": args.epochs}
    for judged in (True, False):
        tag = "judged" if judged else "network_only"
        step(judged)
        ts, (r85, res, choices, look) = timed(lambda: step(judged), max(1, min(args.steps, 3)),
                                              "warm-started sweep (%s)" % tag)
        t = float(np.mean(ts))
        its = [look + r["iterations"] for r in res]
        its.insert(i85, r85["iterations"])
        out[tag] = {"step_ms": round(t * 1e3, 3), "vs_uniform_sweep": round(step_s / t, 3),
                    "iterations": its, "choices": choices, "look_ahead_updates": look,
                    "max_iterations_uniform": max(iters_uniform), "max_iterations_warm": max(its)}
    return out


def relabelled_sweep(args, pr, ctx, dg, problems, path, tau, norm, max_iter, N, E, step_s, seq_s, ranks_b,
                     torch, np):
    """The same sweep and sequential solves on the graph in out-degree order (pr_relabel, timed on
    its own; not part of the headline numbers), the ranks mapped back and compared."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dh, perm = dg.relabelled(ctx)
    torch.cuda.synchronize()
    relabel_ms = (time.perf_counter() - t0) * 1e3
    if args.seg_len:
        dh.prepare_segmented(ctx, seg_len=args.seg_len)
    else:
        dh.prepare(ctx)
    log("relabelled by out-degree in %.1f ms" % relabel_ms)
    if path == "series":
        sweep = lambda: pr.pull_sweep(ctx, dh, problems)  # noqa: E731
    else:
        prec = pr.PR_MIXED if path == "batch_mixed" else pr.PR_FP64
        sweep = lambda: pr.pull_batch(ctx, dh, problems, precision=prec)  # noqa: E731
    seq = lambda: [pr.pull(ctx, dh, alpha=p["alpha"], tau=tau, norm=norm, max_iter=max_iter,  # noqa: E731
                           precision=pr.PR_FP64) for p in problems]
    sweep()
    ts, res = timed(sweep, min(args.steps, 3), "step (batched sweep, degree order)")
    seq()
    ts_seq, _ = timed(seq, 1, "sequential fp64 sweep, degree order")
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    pr.pull(ctx, dh, alpha=0.85, tau=tau, norm=norm, max_iter=max_iter, precision=pr.PR_FP64)
    ctx.set_option("timing", 0)
    n64, ms64 = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F64)
    back = [pr.unpermute(ctx, perm, r["ranks"]) for r in res]
    step = float(np.mean(ts))
    return {"relabel_ms": round(relabel_ms, 2), "batched_sweep_ms": round(step * 1e3, 3),
            "sequential_fp64_ms": round(float(np.mean(ts_seq)) * 1e3, 3),
            "speedup_vs_sequential_fp64": round(float(np.mean(ts_seq)) / step, 3),
            "vs_generated_labels": {"batched_sweep": round(step_s / step, 3),
                                    "sequential_fp64": round(seq_s / float(np.mean(ts_seq)), 3)},
            "iterations": [r["iterations"] for r in res],
            "max_l1_vs_generated_labels": max(pr.l1_distance(ctx, a, b) for a, b in zip(back, ranks_b)),
            "plain_fp64_update": roofline("k_update<double>", single_update_bytes(N, E, 8), ms64 / n64 * 1e-3, n64,
                                          None) if n64 else None}


# ------------------------------------------------------------------ the small configuration

def run_small(args, pr, gg, np, torch):
    g = gg.workload_c1()
    N, E = g.N, g.E
    ctx = pr.Context(0)
    dg = pr.DeviceGraph.from_host(g, 0)
    dg.prepare(ctx)

    def solve():
        return pr.pull(ctx, dg, alpha=0.85, tau=1e-6, norm=pr.PR_L1, max_iter=500)

    for _ in range(args.warmup):
        solve()
    ts, res = timed(solve, args.steps, "solve")
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    solve()
    ctx.set_option("timing", 0)
    n64, ms64 = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F64)
    step_s = float(np.mean(ts))
    line = base_line("small configuration: float64 solve time (alpha=0.85, tau=1e-6, L1) on Erdos-Renyi N=10,000",
                     round(step_s * 1e6, 2), "us", args, step_s * 1e3, "f64",
                     {"workload": "Erdos-Renyi N=10,000, average out-degree 8, 5% forced dangling, no self-loops, "
                                  "seed 1; alpha=0.85, tau=1e-6, L1, uniform start, max_iter 500", "N": N, "E": E},
                     higher=False)
    line["small"] = {"iterations": res["iterations"], "us_per_update": round(step_s * 1e6 / res["iterations"], 2),
                     "update_kernel_us": round(1e3 * ms64 / n64, 2) if n64 else None,
                     "solve_us_min_median": [round(min(ts) * 1e6, 2), round(float(np.median(ts)) * 1e6, 2)],
                     "note": "launch- and latency-bound (working set < 1 MB): no roofline claim"}
    if not args.no_cpu:
        import oracle
        nt = oracle.max_threads()
        out = {}
        for threads in (nt, 1):
            tt = []
            for _ in range(5):
                t0 = time.perf_counter()
                oracle.pagerank_graph(g, alpha=0.85, tau=1e-6, norm=oracle.L1, max_iter=500, threads=threads)
                tt.append(time.perf_counter() - t0)
            out[threads] = float(np.mean(tt))
        line["cpu_baseline"] = {"value": round(out[nt] * 1e6, 2), "unit": "us", "cores": nt,
                                "kind": "oracle", "sample": "the whole solve, mean of 5 runs on %d threads; "
                                "one thread: %.2f us; host CPU %s" % (nt, out[1] * 1e6, cpu_model())}
    ctx.close()
    return line


# ------------------------------------------------------------------ tau x norm readout

def run_tau(args, pr, gg, np, torch):
    scale = args.scale or 22
    seed = args.seed if args.seed is not None else 22
    log("generating R-MAT scale %d seed %d" % (scale, seed))
    g = gg.rmat(scale, edge_factor=16, seed=seed)
    N, E = g.N, g.E
    ctx = pr.Context(0)
    dg = pr.DeviceGraph.from_host(g, 0)
    if args.seg_len:
        dg.prepare_segmented(ctx, seg_len=args.seg_len)
    else:
        dg.prepare(ctx)
    rows = []
    total = {pr.PR_FP64: 0.0, pr.PR_MIXED: 0.0}
    for norm in (pr.PR_L1, pr.PR_L2, pr.PR_LINF):
        for tau in gg.TAU_DECADES:
            res = {}
            for prec in (pr.PR_FP64, pr.PR_MIXED):
                def solve():
                    return pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm, precision=prec)
                solve()
                ts, out = timed(solve, args.steps, "tau %.0e norm %d prec %d" % (tau, norm, prec))
                res[prec] = (float(np.mean(ts)), out)
                total[prec] += float(np.mean(ts))
            f, m = res[pr.PR_FP64][1], res[pr.PR_MIXED][1]
            # ablation: the float32 phase alone, to tau or max_iter (the paper's sensitivity limits)
            a = pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm, precision=pr.PR_FP32)
            rows.append({"tau": tau, "norm": norm, "fp64_iterations": f["iterations"],
                         "fp32_only_iterations": a["iterations"], "fp32_only_converged": bool(a["converged"]),
                         "fp64_ms": round(res[pr.PR_FP64][0] * 1e3, 3),
                         "mixed_iterations": [m["fp32_iters"], m["fp64_iters"]],
                         "mixed_ms": round(res[pr.PR_MIXED][0] * 1e3, 3),
                         "mixed_vs_fp64_l1": pr.l1_distance(ctx, m["ranks"], f["ranks"]),
                         "mixed_vs_fp64_linf": float((m["ranks"] - f["ranks"]).abs().max())})
    # the same float64 readout from one solve: rank snapshots at every (tau, norm) pair as the
    # solve to the last of them (1e-10 in L1) runs; each is the ranks of the separate solve
    pairs = [(tau, norm) for norm in (pr.PR_L1, pr.PR_L2, pr.PR_LINF) for tau in gg.TAU_DECADES]

    def snap_solve():
        return pr.pull_snapshots(ctx, dg, pairs, alpha=0.85, tau=1e-10, norm=pr.PR_L1)
    snap_solve()
    ts, snap = timed(snap_solve, args.steps, "snapshots of %d (tau, norm) pairs" % len(pairs))
    by_pair = {(r["tau"], r["norm"]): r["fp64_iterations"] for r in rows}
    snapshots = {"pairs": len(pairs), "ms": round(float(np.mean(ts)) * 1e3, 3),
                 "separate_fp64_solves_ms": round(total[pr.PR_FP64] * 1e3, 3),
                 "speedup": round(total[pr.PR_FP64] / float(np.mean(ts)), 2), "solve_iterations": snap["iterations"],
                 "iterations_as_separate_solves": all(snap["snap_iter"][i] == by_pair[q] for i, q in enumerate(pairs))}
    one = pr.pull(ctx, dg, alpha=0.85, tau=1e-6, norm=pr.PR_L2)
    snapshots["ranks_as_separate_solve_1e-6_L2"] = bool(torch.equal(snap["snapshots"][pairs.index((1e-6, pr.PR_L2))],
                                                                    one["ranks"]))
    del snap, one
    # sections 4-5 checks per arithmetic and norm, tolerances in decreasing order: the onset of the
    # sensitivity issue (an abrupt jump to max_iter) and the single-iteration stops.  The
    # float32-only ablation continues to tau = 1e-11 and 1e-12.
    from paper_2108_02997_amd import report
    extra = []
    for norm in (pr.PR_L1, pr.PR_L2, pr.PR_LINF):
        for tau in (1e-11, 1e-12):
            a = pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm, precision=pr.PR_FP32)
            extra.append({"tau": tau, "norm": norm, "fp32_only_iterations": a["iterations"],
                          "fp32_only_converged": bool(a["converged"])})
    checks = {}
    for label, count in (("fp64", lambda r: r["fp64_iterations"]), ("mixed", lambda r: sum(r["mixed_iterations"])),
                         ("fp32_only", lambda r: r["fp32_only_iterations"])):
        checks[label] = {}
        for norm, name in ((pr.PR_L1, "L1"), (pr.PR_L2, "L2"), (pr.PR_LINF, "Linf")):
            seq = [r for r in rows if r["norm"] == norm]
            if label == "fp32_only":
                seq += [r for r in extra if r["norm"] == norm]
            seq.sort(key=lambda r: -r["tau"])
            its = [count(r) for r in seq]
            onset = report.sensitivity(its, 500)
            checks[label][name] = {"taus": [r["tau"] for r in seq], "iterations": its,
                                   "sensitivity_onset_tau": seq[onset]["tau"] if onset is not None else None,
                                   "single_iteration_taus": [seq[i]["tau"] for i in report.single_iteration(its)]}
    # the single-vector updates, timed per launch over one float64 and one mixed solve
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    ref = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=pr.PR_L1, precision=pr.PR_FP64)
    pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=pr.PR_LINF, precision=pr.PR_MIXED)
    ctx.set_option("timing", 0)
    n64, ms64 = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F64)
    n32, ms32 = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F32)
    t_ref = [r for r in rows if r["tau"] == 1e-10 and r["norm"] == pr.PR_L1][0]["fp64_ms"] * 1e-3
    line = base_line("tau x norm readout (section 3): iterations and time to each stop, float64 vs mixed; GTEPS "
                     "of the float64 solve to tau=1e-10 (L1)", round(E * ref["iterations"] / t_ref / 1e9, 3),
                     "GTEPS", args, t_ref * 1e3, "f64 | f32+f64",
                     {"workload": "R-MAT scale %d, edge factor 16, (.57,.19,.19,.05), seed %d, alpha=0.85, "
                                  "tau=1e-3..1e-10 x {L1,L2,Linf}, max_iter 500" % (scale, seed), "N": N, "E": E})
    seg = bool(args.seg_len)
    line["config"]["layout"] = ("source-segmented, %d ids per segment" % args.seg_len) if seg else "plain"
    line["roofline"] = roofline("segmented float64 update" if seg else "k_update<double>",
                                single_update_bytes(N, E, 8), ms64 / n64 * 1e-3, n64, None)
    line["fp32_update"] = roofline("segmented float32 update" if seg else "k_update<float>",
                                   single_update_bytes(N, E, 4), ms32 / n32 * 1e-3, n32, None)
    line["readout"] = rows
    line["fp32_only_below_1e-10"] = extra
    line["iteration_checks"] = checks
    line["snapshots"] = snapshots
    # locality of the plain update (no segmented layout): the same graph as generated, under a
    # seeded random relabelling (the stress case) and in out-degree order (hot sources
    # contiguous); update times of one float64 (L1) and one mixed (Linf) solve each, and the
    # float64 ranks mapped back to the generated ids
    locality = {}
    dplain = dg
    if seg:
        dplain = pr.DeviceGraph.from_host(g, 0).prepare(ctx)
    for name in ("as_generated", "random_relabel", "degree_order"):
        relabel_ms = None
        if name == "as_generated":
            perm, dh = None, dplain
        elif name == "random_relabel":
            perm = gg.permutation(N, seed + 7)
            dh = pr.DeviceGraph.from_host(gg.relabel(g, perm), 0).prepare(ctx)
        else:
            # the library's own relabelling (pr_relabel), timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dh, perm_t = dg.relabelled(ctx)
            torch.cuda.synchronize()
            relabel_ms = round((time.perf_counter() - t0) * 1e3, 2)
            perm = perm_t.cpu().numpy()
            dh.prepare(ctx)
        ctx.reset_stats()
        ctx.set_option("timing", 1)
        r64 = pr.pull(ctx, dh, alpha=0.85, tau=1e-10, norm=pr.PR_L1, precision=pr.PR_FP64)
        pr.pull(ctx, dh, alpha=0.85, tau=1e-10, norm=pr.PR_LINF, precision=pr.PR_MIXED)
        ctx.set_option("timing", 0)
        a64, b64 = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F64)
        a32, b32 = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F32)
        back = r64["ranks"] if perm is None else r64["ranks"][torch.from_numpy(perm.astype(np.int64)).cuda()]
        locality[name] = {"f64_update_us": round(1e3 * b64 / a64, 1), "f32_update_us": round(1e3 * b32 / a32, 1),
                          "f64_iterations": r64["iterations"],
                          "f64_frac_of_peak": round(single_update_bytes(N, E, 8) / (b64 / a64 * 1e-3) / 1e9
                                                    / HBM_PEAK_GBS, 4),
                          "l1_vs_as_generated": pr.l1_distance(ctx, back, ref["ranks"])}
        if relabel_ms is not None:
            locality[name]["relabel_ms"] = relabel_ms
        if perm is not None:
            del dh
            torch.cuda.empty_cache()
    line["locality"] = locality
    line["sum_ms"] = {"fp64": round(total[pr.PR_FP64] * 1e3, 2), "mixed": round(total[pr.PR_MIXED] * 1e3, 2)}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline([g], args.cpu_seconds, "the full graph")
    ctx.close()
    return line


# ------------------------------------------------------------------ many graphs, one launch

def run_multi(args, pr, gg, np, torch):
    specs = gg.many_graph_specs()
    log("generating %d graphs" % len(specs))
    hosts = [gg.make_spec_graph(s) for s in specs]
    ctx = pr.Context(0)
    graphs = [pr.DeviceGraph.from_host(h, 0) for h in hosts]
    probs = [dict(alpha=s["alpha"], tau=s["tau"], norm=s["norm"], max_iter=500) for s in specs]
    t = time.time()
    for dg in graphs:
        dg.prepare(ctx)
    torch.cuda.synchronize()
    prep_ms = (time.time() - t) * 1e3
    t = time.time()
    tuned = [dg.autotune(ctx) for dg in graphs]
    tune_s = time.time() - t
    log("autotuned %d graphs in %.1f s" % (len(graphs), tune_s))
    ws = torch.empty(ctx.lib.pr_multi_workspace_bytes(len(graphs), pr.multi_problems(ctx, graphs, probs)[0]),
                     dtype=torch.uint8, device="cuda")

    # outputs allocated once, as a caller reusing its buffers would
    ranks_m = [torch.empty(h.N, dtype=torch.float64, device="cuda") for h in hosts]
    ranks_q = [torch.empty(h.N, dtype=torch.float64, device="cuda") for h in hosts]

    def one_launch():
        return pr.pull_multi(ctx, graphs, probs, workspace=ws, ranks=ranks_m)

    def sequential():
        return [pr.pull(ctx, dg, ranks=r, **p) for dg, p, r in zip(graphs, probs, ranks_q)]

    sequential()
    seq_ts, seq_res = timed(sequential, max(1, args.seq_reps), "64 sequential solves")
    for i in range(args.warmup):
        one_launch()
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    ts, res = timed(one_launch, args.steps, "one persistent launch")
    ctx.set_option("timing", 0)
    nk, msk = ctx.stats(pr._lib.PR_KERNEL_MULTI)
    step_s = float(np.mean(ts))
    edges = sum(h.E * r["iterations"] for h, r in zip(hosts, res))
    alg = sum(single_update_bytes(h.N, h.E, 8) * r["iterations"] for h, r in zip(hosts, res))
    line = base_line("uneven batch of 64 graphs: aggregate GTEPS of one persistent launch vs 64 sequential solves",
                     round(edges / step_s / 1e9, 3), "GTEPS", args, step_s * 1e3, "f64",
                     {"workload": "64 seeded graphs (seed 1000): N log-uniform in [1e3,1e6], even R-MAT / odd "
                                  "Erdos-Renyi, degree {4,8,16,32}, alpha {.75,.85,.95}, tau {1e-6,1e-8,1e-10}, "
                                  "norm {L1,L2,Linf}; autotuned", "graphs": len(hosts),
                      "sum_N": sum(h.N for h in hosts), "sum_E": sum(h.E for h in hosts)})
    traffic = read_traffic("multi_64graphs", source_digest([CSRC + "multi.hip", CSRC + "multi.h", CSRC + "device.h",
                                                           CSRC + "internal.h"]))
    line["roofline"] = roofline("k_multi (whole solve)", alg, msk / nk * 1e-3, nk, traffic)
    line["multi"] = {"sequential_ms": round(float(np.mean(seq_ts)) * 1e3, 3),
                     "speedup_vs_sequential": round(float(np.mean(seq_ts)) / step_s, 3),
                     "iterations": [r["iterations"] for r in res],
                     "same_iterations_as_sequential": sum(int(a["iterations"] == b["iterations"])
                                                          for a, b in zip(res, seq_res)),
                     "max_l1_vs_sequential": max(pr.l1_distance(ctx, a["ranks"], b["ranks"])
                                                 for a, b in zip(res, seq_res)),
                     "prep_ms": round(prep_ms, 2), "autotune_s": round(tune_s, 2),
                     "tuned_mid_deg": [t["mid_deg"] for t in tuned], "tuned_grid": [t["grid"] for t in tuned],
                     "tuned_tile": [t["tile"] for t in tuned], "tuned_tile_batch": [t["tile_batch"] for t in tuned],
                     "tuned_mid_deg_batch": [t["mid_deg_batch"] for t in tuned],
                     "tuned_grid_batch_factor": [t["grid_batch_factor"] for t in tuned]}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(hosts, args.cpu_seconds, "all 64 graphs")
    ctx.close()
    return line


# ------------------------------------------------------------------ sections 3 and 4 over many graphs

def run_norms(args, pr, gg, np, torch):
    from paper_2108_02997_amd import report
    specs = gg.many_graph_specs()
    log("generating %d graphs" % len(specs))
    hosts = [gg.make_spec_graph(s) for s in specs]
    ctx = pr.Context(0)
    graphs = [pr.DeviceGraph.from_host(h, 0) for h in hosts]
    for dg in graphs:
        dg.prepare(ctx)
        dg.autotune(ctx)
    alpha = 0.85
    # section 3: alpha = 0.85, tau = 1e-6, each error function; per graph the mean of `steps`
    # timed solves after one untimed one (the paper times 5 runs and takes the AM)
    it3 = np.zeros((len(graphs), 3))
    ms3 = np.zeros((len(graphs), 3))
    for n in (1, 2, 3):
        for i, dg in enumerate(graphs):
            def solve():
                return pr.pull(ctx, dg, alpha=alpha, tau=1e-6, norm=n)
            solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                out = solve()
            torch.cuda.synchronize()
            ms3[i, n - 1] = (time.perf_counter() - t0) / args.steps * 1e3
            it3[i, n - 1] = out["iterations"]
        log("section 3, norm %d: %d iterations over the graphs" % (n, int(it3[:, n - 1].sum())))
    # the same 64 solves as one persistent launch per error function
    batch_ms, same = [], 0
    for n in (1, 2, 3):
        probs = [dict(alpha=alpha, tau=1e-6, norm=n, max_iter=500)] * len(graphs)
        pr.pull_multi(ctx, graphs, probs)
        ts, res = timed(lambda: pr.pull_multi(ctx, graphs, probs), args.steps, "one launch, norm %d" % n)
        batch_ms.append(round(float(np.mean(ts)) * 1e3, 3))
        same += sum(int(r["iterations"] == k) for r, k in zip(res, it3[:, n - 1].astype(int)))
    # section 4: one traced solve per graph to the smallest tolerance in L1 (the largest of the
    # three errors, so every (tau, norm) stop lies on the trace), all graphs in one launch
    taus = gg.tau_sweep_21()
    probs = [dict(alpha=alpha, tau=min(taus), norm=1, max_iter=500)] * len(graphs)
    t0 = time.perf_counter()
    res = pr.pull_multi(ctx, graphs, probs, trace=True)
    torch.cuda.synchronize()
    sweep_ms = (time.perf_counter() - t0) * 1e3
    Y = np.stack([report.stops(r["trace"].cpu().numpy(), taus) for r in res], axis=1)  # [tau][graph][norm]
    # sections 4-5 checks per graph and norm; a stop the traced solve never reached halted at the
    # limit and counts as max_iter iterations, as the paper's charts show it
    onsets = [report.sensitivity(Y[:, gi, :], 500) for gi in range(len(graphs))]
    Y = np.where(Y == 0, 500, Y)
    edges = float(sum(h.E * r["iterations"] for h, r in zip(hosts, res)))
    line = base_line("sections 3-4 over 64 graphs: GM-RATIO of iterations, Linf vs L1 (alpha=0.85, tau=1e-6)",
                     round(report.composite(it3, 0)["GM-RATIO"][2], 4), "ratio", args, float(np.sum(ms3[:, 0])),
                     "f64", {"workload": "64 seeded graphs (seed 1000) as in --workload multi, every graph at "
                                         "alpha=0.85; section 3 at tau=1e-6 for L1/L2/Linf; section 4 over the 21 "
                                         "tolerances 1 ... 1e-10 read off one traced solve per graph",
                             "graphs": len(hosts), "sum_E": sum(h.E for h in hosts)}, higher=False)
    line["section3"] = {
        "iterations_mean": [round(x, 3) for x in it3.mean(axis=0)],
        "time_ms_sum_sequential": [round(x, 3) for x in ms3.sum(axis=0)],
        "time_ms_one_launch": batch_ms,
        "one_launch_same_iterations": "%d of %d" % (same, 3 * len(graphs)),
        "table_3_1_times": {"baseline_L1": report.composite(ms3, 0), "baseline_Linf": report.composite(ms3, 2)},
        "table_3_2_iterations": {"baseline_L1": report.composite(it3, 0), "baseline_Linf": report.composite(it3, 2)},
    }
    line["section4"] = {
        "taus": list(taus),
        "mean_iterations_per_tau": [[round(float(x), 3) for x in Y[i].mean(axis=0)] for i in range(len(taus))],
        "nested_AM_vs_L1": report.nested(Y, 0, "AM"), "nested_GM_vs_L1": report.nested(Y, 0, "GM"),
        "single_iteration_stops": [[int(x) for x in (Y[i] == 1).sum(axis=0)] for i in range(len(taus))],
        "graphs_with_sensitivity_issue": [sum(o[j] is not None for o in onsets) for j in range(3)],
        "sensitivity_onset_taus": [[taus[o[j]] for o in onsets if o[j] is not None] for j in range(3)],
        "traced_launch_ms": round(sweep_ms, 3), "traced_launch_GTEPS": round(edges / sweep_ms / 1e6, 2),
    }
    # section 5's single-iteration convergence on a large road-like graph: a 2048 x 2048 lattice,
    # one traced solve (L1, the largest of the three errors) read at the 21 tolerances per norm
    lat = gg.grid2d(2048, 2048)
    dl = pr.DeviceGraph.from_host(lat, 0).prepare(ctx)
    rl = pr.pull(ctx, dl, alpha=alpha, tau=min(taus), norm=pr.PR_L1, max_iter=500, trace=True)
    S = report.stops(rl["trace"].cpu().numpy(), taus)  # [tau][norm]
    onsets = report.sensitivity(S, 500)
    singles = report.single_iteration(S)
    line["road_like"] = {"graph": "2048 x 2048 lattice (each cell linked both ways to its 4 neighbours)",
                         "N": lat.N, "E": lat.E, "alpha": alpha, "taus": list(taus)}
    for j, name in enumerate(("L1", "L2", "Linf")):
        line["road_like"][name] = {"iterations": [int(x) for x in S[:, j]],
                                   "single_iteration_taus": [taus[i] for i in singles[j]],
                                   "sensitivity_onset_tau": taus[onsets[j]] if onsets[j] is not None else None}
    del dl
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(hosts, args.cpu_seconds, "all 64 graphs")
    ctx.close()
    return line


# ------------------------------------------------------------------ learned warm start

def run_warmstart(args, pr, gg, np, torch):
    from paper_2108_02997_amd import warmstart as wsm
    ctx = pr.Context(0)
    model = wsm.WarmStart(ctx, seed=0)
    train_alphas = [0.5, 0.55, 0.6, 0.65, 0.7, 0.75, 0.8, 0.85, 0.9, 0.95, 0.99]
    samples = []
    t = time.time()
    for s in range(20):
        h = gg.rmat(20, edge_factor=16, seed=2000 + s)
        dg = pr.DeviceGraph.from_host(h, 0)
        samples += model.make_samples(dg, train_alphas)
        del dg
    label_s = time.time() - t
    log("labelled %d samples in %.1f s" % (len(samples), label_s))
    torch.cuda.synchronize()
    t = time.time()
    hist = model.train(samples, epochs=args.epochs, lr=3e-3)
    torch.cuda.synchronize()
    train_s = time.time() - t
    log("trained %d epochs in %.1f s, loss %.4f -> %.4f" % (args.epochs, train_s, hist[0], hist[-1]))
    del samples
    torch.cuda.empty_cache()

    scale = args.scale or 24
    seeds = [args.seed] if args.seed is not None else [3000, 3001, 3002]
    tau, norm = 1e-10, pr.PR_LINF
    rows = []
    for seed in seeds:
        log("evaluation graph: R-MAT scale %d seed %d" % (scale, seed))
        g = gg.rmat(scale, edge_factor=16, seed=seed)
        dg = pr.DeviceGraph.from_host(g, 0)
        dg.prepare(ctx)
        r85 = pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm)
        for alpha in (0.90, 0.95, 0.99):
            def uni():
                return pr.pull(ctx, dg, alpha=alpha, tau=tau, norm=norm)

            def from85():
                return pr.pull(ctx, dg, alpha=alpha, tau=tau, norm=norm, init=r85["ranks"])

            def frommlp():
                r0 = model.propose(dg, r85["ranks"], alpha)
                return pr.pull(ctx, dg, alpha=alpha, tau=tau, norm=norm, init=r0)

            def judged():
                r0, name, _, steps, _ = model.start(dg, r85["ranks"], alpha, norm=norm)
                out = pr.pull(ctx, dg, alpha=alpha, tau=tau, norm=norm, init=r0)
                out["iterations_total"] = steps + out["iterations"]
                out["choice"] = name
                return out

            row = {"graph_seed": seed, "alpha": alpha}
            ref = None
            for tag, fn in (("uniform", uni), ("r085", from85), ("mlp", frommlp), ("judged", judged)):
                fn()
                ts, out = timed(fn, args.steps, "seed %d alpha %.2f %s" % (seed, alpha, tag))
                row[tag + "_ms"] = round(float(np.mean(ts)) * 1e3, 3)
                row[tag + "_iterations"] = out.get("iterations_total", out["iterations"])
                if tag == "uniform":
                    ref = out["ranks"]
                else:
                    row[tag + "_linf_vs_uniform"] = float((out["ranks"] - ref).abs().max())
                if tag == "judged":
                    row["judged_choice"] = out["choice"]
            rows.append(row)
        if seed != seeds[-1]:
            del dg, r85
            torch.cuda.empty_cache()
    t_uni = sum(r["uniform_ms"] for r in rows)
    t_mlp = sum(r["mlp_ms"] for r in rows)
    line = base_line("learned warm start: time to tau=1e-10 (Linf) from the network's start (features and inference "
                     "included) against the uniform start, summed over alpha = 0.90, 0.95, 0.99 and the "
                     "evaluation graphs",
                     round(t_uni / t_mlp, 3), "x", args, t_mlp, "f64 solve; f32 weights, bf16 activations",
                     {"workload": "train: 20 R-MAT scale-20 graphs (seeds 2000-2019), alpha in {.50..,.95,.99}, "
                                  "labels at tau=1e-12 (L1); evaluate: unseen R-MAT scale %d, seeds %s"
                                  % (scale, ", ".join(str(x) for x in seeds)),
                      "N": g.N, "E": g.E, "tau": tau, "norm": "Linf"})
    line["warm_start"] = {"rows": rows, "train_s": round(train_s, 2), "label_s": round(label_s, 2),
                          "epochs": args.epochs, "loss_first_last": [hist[0], hist[-1]],
                          "iterations_sum": {k: sum(r[k + "_iterations"] for r in rows)
                                             for k in ("uniform", "r085", "mlp", "judged")},
                          "judged_vs_uniform_time": round(t_uni / sum(r["judged_ms"] for r in rows), 3)}
    # dominant kernel of the timed solves: the float64 update, event-timed per launch
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    pr.pull(ctx, dg, alpha=0.95, tau=tau, norm=norm, init=model.propose(dg, r85["ranks"], 0.95))
    ctx.set_option("timing", 0)
    n64, ms64 = ctx.stats(pr._lib.PR_KERNEL_UPDATE_F64)
    if n64:
        line["roofline"] = roofline("k_update<double>", single_update_bytes(g.N, g.E, 8), ms64 / n64 * 1e-3, n64, None)
    # the network's inference on the matrix cores: 2 (32*6 + 32*32) flops per vertex in the two
    # hidden layers (the bias as a sixth input), priced against the dense float32 MFMA peak
    feat, _ = wsm.features(ctx, dg, r85["ranks"], 0.95)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wsm.forward(ctx, model.W, feat)
    e0.record()
    for _ in range(5):
        wsm.forward(ctx, model.W, feat)
    e1.record()
    torch.cuda.synchronize()
    fwd_s = e0.elapsed_time(e1) / 5 * 1e-3
    flops = 2.0 * (32 * 6 + 32 * 32) * g.N
    line["mlp_forward"] = {"kernel": "k_mlp_forward (inference, N=%d)" % g.N, "bound": "mfma",
                           "achieved": round(flops / fwd_s / 1e12, 2), "peak": FP32_MFMA_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(flops / fwd_s / 1e12 / FP32_MFMA_PEAK_TFLOPS, 4),
                           "avg_launch_us": round(fwd_s * 1e6, 1), "flops_per_vertex": 2 * (32 * 6 + 32 * 32)}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline([g], args.cpu_seconds, "the evaluation graph")
    ctx.close()
    return line


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["sweep", "small", "tau", "multi", "norms", "warmstart"], default="sweep")
    ap.add_argument("--scale", type=int, default=None, help="R-MAT scale (default: 24, or 22 for --workload tau)")
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-relabel", action="store_true", help="skip the sweep on the out-degree-ordered graph")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--calibrate", action="store_true", help="accepted for older command lines; the 1 GiB copy "
                    "that calibrates the memory counters now always runs")
    ap.add_argument("--path", choices=["series", "batch_mixed", "batch_fp64"], default="series",
                    help="the timed sweep: one float64 iteration for all columns (power series in the damping "
                         "factor, default), the batched mixed-precision columns, or batched float64 columns")
    ap.add_argument("--seq-reps", type=int, default=2, help="timed repetitions of the sequential FP64 baseline")
    ap.add_argument("--epochs", type=int, default=20, help="training epochs of the warm-start network")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-started sweep")
    ap.add_argument("--seg-len", type=int, default=1 << 19, help="source ids per segment of the source-segmented "
                    "layout used by the sweep and tau workloads' single-vector updates (0: the plain update)")
    ap.add_argument("--warm-graphs", type=int, default=8, help="training graphs of the warm-started sweep's network")
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
    run = {"sweep": run_sweep, "small": run_small, "tau": run_tau, "multi": run_multi, "norms": run_norms,
           "warmstart": run_warmstart}[args.workload]
    line = run(args, pr, gg, np, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
