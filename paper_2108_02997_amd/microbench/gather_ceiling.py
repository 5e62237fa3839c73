#!/usr/bin/env python3
"""Memory-access ceiling of one pull update on a graph, measured with gather_ceiling.hip.

Runs, on the in-edge index array of a seeded R-MAT graph (default: scale 24, seed 24, the
benchmark's graph), the bare accesses of an update -- the index stream alone, a float64 or float32
scalar per entry, a 16/32/48/64-byte row per entry (48-byte rows also as 4 lanes x 12 bytes and as
3 of 4 lanes x 16 bytes) -- and, for comparison, the update kernels of
libprpull.so on the same graph (event-timed, pr_get_stats).  Prints one JSON line.
Not part of the solver; the oracle is not used.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

# gc_run kinds by bytes fetched per entry (float32, float64, 16/32/48/64-byte rows)
ROW_KINDS = {4: 1, 8: 0, 16: 3, 32: 4, 48: 6, 64: 5}


def load():
    """The measurement library (built by paper_2108_02997_amd/build.py)."""
    lib = ctypes.CDLL(os.path.join(HERE, "libgather_ceiling.so"))
    lib.gc_run.restype = ctypes.c_int
    lib.gc_run.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_int, ctypes.c_void_p]
    return lib


def bare_gather_ms(lib, idx, N: int, row_bytes: int, reps: int = 5, grid: int = 4096) -> float:
    """HIP-event average of the bare gather of one `row_bytes` row per entry of the device int32
    index array `idx` (values < N) from a random table, on torch's current stream."""
    import torch
    kind = ROW_KINDS[row_bytes]
    E = idx.numel()
    table = torch.rand(N * max(row_bytes, 8) // 4, dtype=torch.float32, device=idx.device)
    out = torch.empty(grid * 256, dtype=torch.float64, device=idx.device)
    stream = torch.cuda.current_stream().cuda_stream

    def once():
        rc = lib.gc_run(kind, idx.data_ptr(), E, table.data_ptr(), out.data_ptr(), grid, stream)
        if rc != 0:
            raise RuntimeError("gc_run(%d) failed: %d" % (kind, rc))

    once()
    once()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--seed", type=int, default=24)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()

    import numpy as np
    import torch

    import graphgen as gg
    import paper_2108_02997_amd as pr

    lib = ctypes.CDLL(os.path.join(HERE, "libgather_ceiling.so"))
    lib.gc_run.restype = ctypes.c_int
    lib.gc_run.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_int, ctypes.c_void_p]
    g = gg.rmat(args.scale, edge_factor=16, seed=args.seed)
    N, E = g.N, g.E
    print("graph N=%d E=%d" % (N, E), file=sys.stderr, flush=True)
    assert int(g.idx.max()) < N and int(g.idx.min()) >= 0
    idx = torch.from_numpy(np.ascontiguousarray(g.idx)).cuda()
    grid = 4096
    out = torch.empty(grid * 256, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream

    def run(kind, table, label, useful_bytes):
        for _ in range(2):
            rc = lib.gc_run(kind, idx.data_ptr(), E, table.data_ptr() if table is not None else None, out.data_ptr(),
                            grid, stream)
            if rc != 0:
                raise RuntimeError("gc_run(%d) failed: %d" % (kind, rc))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            lib.gc_run(kind, idx.data_ptr(), E, table.data_ptr() if table is not None else None, out.data_ptr(), grid,
                       stream)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.reps
        print("%-28s %.3f ms" % (label, ms), file=sys.stderr, flush=True)
        return {"what": label, "ms": round(ms, 4), "useful_GBps": round(useful_bytes / ms / 1e6, 1)}

    rows = [run(2, None, "index stream", 4 * E)]
    y64 = torch.rand(N, dtype=torch.float64, device="cuda")
    rows.append(run(0, y64, "float64 per entry", 12 * E))
    rows.append(run(1, y64.float(), "float32 per entry", 8 * E))
    del y64
    for q, kind in ((1, 3), (2, 4), (3, 6), (4, 5)):
        Y = torch.rand(N * 4 * q, dtype=torch.float32, device="cuda")
        rows.append(run(kind, Y, "%d-byte row per entry" % (16 * q), (4 + 16 * q) * E))
        if q == 3:
            rows.append(run(7, Y, "48-byte row, 4 lanes x 12 B", 52 * E))
            rows.append(run(8, Y, "48-byte row, 3 of 4 lanes x 16 B", 52 * E))
        del Y

    # the solver's update kernels on the same graph, event-timed per launch
    ctx = pr.Context(0)
    dg = pr.DeviceGraph.from_host(g)
    dg.prepare(ctx)
    kernels = []
    for prec, kind, name in ((pr.PR_FP64, pr._lib.PR_KERNEL_UPDATE_F64, "k_update<double>"),
                             (pr.PR_MIXED, pr._lib.PR_KERNEL_UPDATE_F32, "k_update<float>")):
        pr.pull(ctx, dg, alpha=0.85, tau=1e-30, norm=3, max_iter=6, precision=prec)
        ctx.reset_stats()
        ctx.set_option("timing", 1)
        pr.pull(ctx, dg, alpha=0.85, tau=1e-30, norm=3, max_iter=6, precision=prec)
        ctx.set_option("timing", 0)
        n, ms = ctx.stats(kind)
        kernels.append({"kernel": name, "us": round(1e3 * ms / n, 1)})
    for K, W in ((1, 1), (2, 2), (4, 4), (8, 8), (11, 12), (16, 16)):
        probs = [dict(alpha=0.85, tau=1e-30, norm=3, max_iter=6)] * K
        pr.pull_batch(ctx, dg, probs, precision=pr.PR_MIXED)
        ctx.reset_stats()
        ctx.set_option("timing", 1)
        pr.pull_batch(ctx, dg, probs, precision=pr.PR_MIXED)
        ctx.set_option("timing", 0)
        n, ms = ctx.stats(pr._lib.batch_kind(True, W))
        kernels.append({"kernel": "k_batch_update<float,%d> (%d columns, %d-byte rows)" % (W, K, 4 * W),
                        "us": round(1e3 * ms / n, 1)})
    ctx.close()
    print(json.dumps({"graph": "R-MAT scale %d seed %d" % (args.scale, args.seed), "N": N, "E": E,
                      "bare_accesses": rows, "update_kernels": kernels}), flush=True)


if __name__ == "__main__":
    main()
