// api_solve.hip -- the C ABI of the single and K-column solves: pr_pull (float64, mixed, float32
// phases), pr_pull_snapshots (pr_pull with rank snapshots at given (tau, norm) pairs) and
// pr_pull_batch (column compaction between chunks, float32 -> float64 hand-over), and the L1
// distance of two rank vectors.
#include <string.h>

#include <algorithm>

#include "api_internal.h"
#include "sweep.h"

extern "C" {

size_t pr_workspace_bytes(int64_t N, int64_t E, int32_t precision, int32_t with_prep) {
  if (bad_graph_sizes(N, E) || (precision != PR_FP64 && precision != PR_MIXED && precision != PR_FP32)) return 0;
  return carve(nullptr, N, E, precision, with_prep != 0).total;
}

int pr_pull(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
            int64_t N, int64_t E, const void *prep, double alpha, double tau, int32_t norm, int32_t max_iter,
            int32_t precision, const double *init, double *ranks, double *norm_trace, void *workspace,
            size_t workspace_bytes, pr_result *out) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !workspace || !out || (E > 0 && !in_indices)) {
    set_error("pr_pull: NULL argument");
    return PR_EINVAL;
  }
  return pull_solve(ctx, stream, in_offsets, in_indices, outdeg, N, E, prep, alpha, tau, norm, max_iter, precision,
                    init, ranks, norm_trace, workspace, workspace_bytes, out);
}

int pr_pull_snapshots(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                      const int32_t *outdeg, int64_t N, int64_t E, const void *prep, double alpha, double tau,
                      int32_t norm, int32_t max_iter, int32_t precision, const double *init, double *ranks,
                      double *norm_trace, int32_t S, const double *snap_tau, const int32_t *snap_norm,
                      double *snaps, int32_t *snap_iter, void *workspace, size_t workspace_bytes, pr_result *out) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !workspace || !out || (E > 0 && !in_indices) || !snap_tau ||
      !snap_norm || !snaps || !snap_iter) {
    set_error("pr_pull_snapshots: NULL argument");
    return PR_EINVAL;
  }
  const SnapRequest r{S, snap_tau, snap_norm, snaps, snap_iter};
  return pull_solve(ctx, stream, in_offsets, in_indices, outdeg, N, E, prep, alpha, tau, norm, max_iter, precision,
                    init, ranks, norm_trace, workspace, workspace_bytes, out, &r);
}

}  // extern "C"

namespace prpull {

// The source-segmented update's arrays (per-segment step over the pair CSR, merge step over the
// merge CSR in place of the plain tiles) from a prep buffer that holds the layout.
static void set_segmented(const pr_ctx *ctx, const PrepHeader &h, const void *pp, bool fp32, IterParams &p) {
  char *base = (char *)const_cast<void *>(pp);
  p.off = (const int32_t *)(base + h.sl.moff_off);
  p.idx = (const int32_t *)(base + h.sl.mpos_off);
  p.poff = (const int32_t *)(base + h.sl.poff_off);
  p.sidx = (const int32_t *)(base + h.sl.sidx_off);
  p.pdesc = (const int4 *)(base + h.sl.pair_part.desc_off);
  p.npdesc = h.sl.pair_part.ndesc;
  p.partial = base + h.sl.part_off;
  // explicit options first, then the autotuner's table, then the defaults
  int64_t pair_mid = ctx->pair_mid_deg, seg_grid = ctx->seg_grid, merge_xcd = ctx->merge_xcd;
  if (ctx->use_tuned) {
    auto it = ctx->tuned_seg.find(seg_signature(h));
    if (it != ctx->tuned_seg.end()) {
      if (!ctx->pair_mid_deg_set) pair_mid = it->second.pair_mid_deg;
      if (!ctx->seg_grid_set) seg_grid = it->second.seg_grid;
      if (!ctx->merge_xcd_set) merge_xcd = it->second.merge_xcd;
    }
  }
  // by default the update kernel's resident count (7 workgroups per CU in float64): measured
  // faster than the per-segment step's own full occupancy of 8, whose extra tiles in flight
  // crowd the segment's slice in L2 (R-MAT scale 24: 1.77 against 1.81 ms per update)
  const int64_t sg = seg_grid > 0 ? seg_grid : ctx->resident[fp32 ? 1 : 0];
  p.pgrid = (int32_t)std::max<int64_t>(1, std::min<int64_t>({(int64_t)p.npdesc, sg, kMaxGrid}));
  p.seg_xcd = (int32_t)ctx->seg_xcd;
  p.merge_xcd = (int32_t)merge_xcd;
  p.pair_mid_deg = (int32_t)pair_mid;
}

// pr_pull after its NULL checks (also the body of the entry point that allocates nothing).
int pull_solve(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
               int64_t N, int64_t E, const void *prep, double alpha, double tau, int32_t norm, int32_t max_iter,
               int32_t precision, const double *init, double *ranks, double *norm_trace, void *workspace,
               size_t workspace_bytes, pr_result *out, const SnapRequest *snaps) {
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  if (!(alpha >= 0.0 && alpha <= 1.0)) {
    set_error("alpha must be in [0, 1], got %g", alpha);
    return PR_EINVAL;
  }
  if (!(tau >= 0.0)) {
    set_error("tau must be >= 0 and not NaN, got %g", tau);
    return PR_EINVAL;
  }
  if (norm < PR_L1 || norm > PR_LINF) {
    set_error("norm must be PR_L1, PR_L2 or PR_LINF, got %d", norm);
    return PR_EINVAL;
  }
  if (max_iter < 1) {
    set_error("max_iter must be >= 1, got %d", max_iter);
    return PR_EINVAL;
  }
  if (precision != PR_FP64 && precision != PR_MIXED && precision != PR_FP32) {
    set_error("precision must be PR_FP64, PR_MIXED or PR_FP32, got %d", precision);
    return PR_EINVAL;
  }
  if (snaps) {
    if (precision == PR_MIXED) {
      set_error("pr_pull_snapshots: precision must be PR_FP64 or PR_FP32 (a mixed solve changes phase)");
      return PR_EINVAL;
    }
    if (snaps->S < 1 || snaps->S > kMaxSnaps) {
      set_error("pr_pull_snapshots: S must be in [1, %d], got %d", kMaxSnaps, snaps->S);
      return PR_EINVAL;
    }
    for (int i = 0; i < snaps->S; ++i)
      if (!(snaps->tau[i] >= 0.0) || snaps->norm[i] < PR_L1 || snaps->norm[i] > PR_LINF) {
        set_error("pr_pull_snapshots: snapshot %d needs tau >= 0 and norm PR_L1, PR_L2 or PR_LINF", i);
        return PR_EINVAL;
      }
  }
  const Layout L = carve(workspace, N, E, precision, prep == nullptr);
  if (workspace_bytes < L.total) {
    set_error("pr_pull: workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  int rc;
  const void *pp = prep;
  if (!prep) {
    rc = prepare_into(ctx, s, in_offsets, N, E, L.prep, &h);
    pp = L.prep;
  } else {
    rc = get_prep(ctx, s, prep, N, E, &h);
  }
  if (rc != PR_OK) return rc;

  PR_HIP(launch_fill_u32(s, (uint32_t *)L.st, sizeof(SolveState) / 4, 0u));
  const std::pair<int32_t, int64_t> ts = tuned_settings(ctx, h);
  const int64_t gcap = ts.second > 0 ? ts.second : ctx->resident[precision == PR_FP64 ? 0 : 1];
  // a prep with the source-segmented layout: the merge step's tiles take the place of the plain
  // update's, the per-segment step runs before it
  const bool seg = ctx->segmented != 0 && h.seg_len > 0;
  const PrepPart &part = seg ? h.sl.merge_part : h.part[0];
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>({(int64_t)part.ndesc, gcap, kMaxGrid}));

  IterParams p{};
  p.off = in_offsets;
  p.idx = in_indices;
  if (seg) set_segmented(ctx, h, pp, precision != PR_FP64, p);
  p.outdeg = outdeg;
  p.desc = (const int4 *)((const char *)pp + part.desc_off);
  p.ndesc = part.ndesc;
  p.N = (int32_t)N;
  p.alpha = alpha;
  p.tau = tau;
  p.norm = norm;
  p.max_iter = max_iter;
  p.st = L.st;
  p.bpart = L.bpart;
  p.hpart = L.hpart;
  p.hubs = (const int4 *)((const char *)pp + part.hub_off);
  p.nhubs = part.nhubs;
  p.grid = (int32_t)grid;
  p.trace = norm_trace;
  p.mid_deg = ts.first;
  if (snaps) {
    SnapTable t{};
    for (int i = 0; i < snaps->S; ++i) {
      t.tau[i] = snaps->tau[i];
      t.norm[i] = snaps->norm[i];
    }
    t.S = snaps->S;
    t.out = snaps->out;
    t.node = -1;
    PR_HIP(hipMemcpyAsync(L.snap, &t, sizeof t, hipMemcpyHostToDevice, s));
    PR_HIP(hipStreamSynchronize(s));  // t is this frame's
    p.snap = L.snap;
  }

  int fp32_iters = 0, fbuf = 0;
  const void *final_y = nullptr;
  bool final_fp32 = false;
  if (precision == PR_MIXED) {
    PR_HIP(launch_init(s, true, outdeg, (int32_t)N, init, L.y32[0], alpha, L.st, L.bpart, kMaxGrid));
    p.phase = 1;
    rc = run_until_stop(ctx, s, update_chunk(ctx, true, grid, p, L.y32[0], L.y32[1]), &L.st->head, max_iter, &fbuf);
    if (rc != PR_OK) return rc;
    fp32_iters = ((LoopHead *)ctx->hstate)->iter;
    if (((LoopHead *)ctx->hstate)->done) {
      final_y = L.y32[fbuf];
      final_fp32 = true;
    } else {
      PR_HIP(launch_convert(s, L.y32[fbuf], L.y64[0], (int32_t)N, L.st));
      p.phase = 2;
      rc = run_until_stop(ctx, s, update_chunk(ctx, false, grid, p, L.y64[0], L.y64[1]), &L.st->head, max_iter,
                          &fbuf);
      if (rc != PR_OK) return rc;
      final_y = L.y64[fbuf];
    }
  } else if (precision == PR_FP32) {
    // the float32 phase alone, stopping like a float64 solve (tau met or max_iter)
    PR_HIP(launch_init(s, true, outdeg, (int32_t)N, init, L.y32[0], alpha, L.st, L.bpart, kMaxGrid));
    p.phase = 0;
    rc = run_until_stop(ctx, s, update_chunk(ctx, true, grid, p, L.y32[0], L.y32[1]), &L.st->head, max_iter, &fbuf);
    if (rc != PR_OK) return rc;
    fp32_iters = ((LoopHead *)ctx->hstate)->iter;
    final_y = L.y32[fbuf];
    final_fp32 = true;
  } else {
    PR_HIP(launch_init(s, false, outdeg, (int32_t)N, init, L.y64[0], alpha, L.st, L.bpart, kMaxGrid));
    p.phase = 0;
    rc = run_until_stop(ctx, s, update_chunk(ctx, false, grid, p, L.y64[0], L.y64[1]), &L.st->head, max_iter, &fbuf);
    if (rc != PR_OK) return rc;
    final_y = L.y64[fbuf];
  }
  PR_HIP(launch_output(s, final_fp32, outdeg, final_y, (int32_t)N, ranks));
  PR_HIP(hipMemcpyAsync(ctx->hstate, L.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
  if (snaps) PR_HIP(hipMemcpyAsync(snaps->iter, L.snap->iter, sizeof(int32_t) * snaps->S, hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  const SolveState &hs = *ctx->hstate;
  out->iterations = hs.head.iter;
  out->converged = hs.converged;
  out->fp32_iters = precision == PR_FP64 ? 0 : fp32_iters;
  out->fp64_iters = hs.head.iter - out->fp32_iters;
  out->final_err[0] = hs.err[0];
  out->final_err[1] = hs.err[1];
  out->final_err[2] = hs.err[2];
  return hs.converged ? PR_OK : PR_NOT_CONVERGED;
}

}  // namespace prpull

extern "C" {

size_t pr_batch_workspace_bytes(int64_t N, int64_t E, int32_t K, int32_t precision, int32_t with_prep) {
  if (bad_graph_sizes(N, E) || K < 1 || K > kMaxCols || (precision != PR_FP64 && precision != PR_MIXED)) return 0;
  return carve_batch(nullptr, N, E, K, precision, with_prep != 0).total;
}

int pr_pull_batch(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                  const int32_t *outdeg, int64_t N, int64_t E, const void *prep, int32_t K, const pr_problem *probs,
                  int32_t precision, const double *const *init, double *const *ranks, double *const *norm_trace,
                  void *workspace, size_t workspace_bytes, pr_result *results) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !probs || !workspace || !results || (E > 0 && !in_indices)) {
    set_error("pr_pull_batch: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  if (K < 1 || K > kMaxCols) {
    set_error("K must be in [1, %d], got %d", kMaxCols, K);
    return PR_EINVAL;
  }
  if (precision != PR_FP64 && precision != PR_MIXED) {
    set_error("precision must be PR_FP64 or PR_MIXED, got %d", precision);
    return PR_EINVAL;
  }
  for (int k = 0; k < K; ++k) {
    const pr_problem &q = probs[k];
    if (!(q.alpha >= 0.0 && q.alpha <= 1.0) || !(q.tau >= 0.0) || q.norm < PR_L1 || q.norm > PR_LINF ||
        q.max_iter < 1 || !ranks[k]) {
      set_error("problem %d: alpha in [0,1], tau >= 0, norm 1..3, max_iter >= 1 and a ranks buffer are required", k);
      return PR_EINVAL;
    }
  }
  const BatchLayout L = carve_batch(workspace, N, E, K, precision, prep == nullptr);
  if (workspace_bytes < L.total) {
    set_error("pr_pull_batch: workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  int rc;
  const void *pp = prep;
  if (!prep) {
    rc = prepare_into(ctx, s, in_offsets, N, E, L.prep, &h);
    pp = L.prep;
  } else {
    rc = get_prep(ctx, s, prep, N, E, &h);
  }
  if (rc != PR_OK) return rc;
  int max_iter = 1;
  for (int k = 0; k < K; ++k) max_iter = std::max(max_iter, probs[k].max_iter);

  const PrepPart &part = h.part[1];
  BatchParams p{};
  p.off = in_offsets;
  p.idx = in_indices;
  p.outdeg = outdeg;
  p.desc = (const int4 *)((const char *)pp + part.desc_off);
  p.ndesc = part.ndesc;
  p.N = (int32_t)N;
  p.nhubs = part.nhubs;
  p.hubs = (const int4 *)((const char *)pp + part.hub_off);
  p.bpart = L.bpart;
  p.hpart = L.hpart;
  p.hacc = L.hacc;
  p.st = L.st;
  p.cols = L.cols;
  // the autotuner's choice for this graph (wave-per-row threshold, workgroups per resident slot)
  const std::pair<int32_t, int32_t> tb = tuned_batch_settings(ctx, h);
  p.mid_deg = tb.first;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1) cus = 1;
  auto grid_of = [&](bool fp32, int kpw) {
    const int64_t res =
        ctx->max_grid > 0 ? ctx->max_grid : (int64_t)cus * batch_blocks_per_cu(fp32, kpw) * (int64_t)tb.second;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>({(int64_t)part.ndesc, res, kMaxGrid}));
  };

  // The running layout: slot i holds original problem orig[i]; `master` keeps every original
  // problem's latest column state on the host.
  int orig[kMaxCols];
  BatchColumn master[kMaxCols];
  memset(master, 0, sizeof master);
  int Kc = K;
  for (int i = 0; i < K; ++i) orig[i] = i;
  // Write the per-slot parameters (slot order) with the given map/ranks choice and wait for the
  // copy, so the pinned staging buffer may be rewritten afterwards.
  auto write_cols = [&](int n, const int *slot_orig, const int *map, bool with_ranks, const bool *rank_sel) -> int {
    BatchCols &hc = *ctx->hcols;
    memset(&hc, 0, sizeof hc);
    for (int i = 0; i < n; ++i) {
      const int k = slot_orig[i];
      hc.alpha[i] = probs[k].alpha;
      hc.tau[i] = probs[k].tau;
      hc.norm[i] = probs[k].norm;
      hc.max_iter[i] = probs[k].max_iter;
      hc.init[i] = init ? init[k] : nullptr;
      hc.ranks[i] = with_ranks && (!rank_sel || rank_sel[i]) ? ranks[k] : nullptr;
      hc.trace[i] = norm_trace ? norm_trace[k] : nullptr;
      hc.map[i] = map ? map[i] : -1;
    }
    PR_HIP(hipMemcpyAsync(L.cols, &hc, sizeof hc, hipMemcpyHostToDevice, s));
    PR_HIP(hipStreamSynchronize(s));
    return PR_OK;
  };
  auto stat_chunk = [&](const ChunkSpec &cs, const std::vector<hipEvent_t> *ev, int did) -> int {
    if (!ev || did <= 0) return PR_OK;
    float ms = 0.f;
    for (int k = 0; k < did && k < cs.count; ++k) {
      PR_HIP(hipEventElapsedTime(&ms, (*ev)[k], (*ev)[k + 1]));
      ctx->stat_ms[cs.kind] += ms;
      ctx->stat_launches[cs.kind] += 1;
      ctx->stat_ms[cs.sub_kind] += ms;
      ctx->stat_launches[cs.sub_kind] += 1;
    }
    return PR_OK;
  };

  const bool mixed = precision == PR_MIXED;
  const bool fp32 = mixed;  // first phase arithmetic
  const bool narrow = ctx->narrow != 0;
  int kp = batch_row_width(Kc, fp32, narrow);
  void *b0 = fp32 ? (void *)L.y32[0] : (void *)L.y64[0];
  void *b1 = fp32 ? (void *)L.y32[1] : (void *)L.y64[1];
  const int kp64 = batch_row_width(K, false, narrow);

  rc = write_cols(Kc, orig, nullptr, false, nullptr);
  if (rc != PR_OK) return rc;
  PR_HIP(launch_fill_u32(s, (uint32_t *)L.st, sizeof(BatchState) / 4, 0u));
  p.K = Kc;
  p.phase = mixed ? 1 : 0;
  p.grid = (int32_t)grid_of(fp32, kp);
  PR_HIP(launch_batch_init(s, fp32, outdeg, (int32_t)N, Kc, kp, b0, L.bpart, kMaxGrid, p, p.phase));

  // ---- first phase, with compaction of the active columns into narrower rows
  int before = 0;
  for (int rounds = 0;; ++rounds) {
    ChunkSpec cs = batch_chunk(ctx, fp32, kp, (unsigned)p.grid, p, b0, b1);
    cs.count = (int)ctx->batch_chunk;
    const std::vector<hipEvent_t> *ev = nullptr;
    rc = run_chunk(ctx, s, cs, &ev);
    if (rc != PR_OK) return rc;
    PR_HIP(hipMemcpyAsync(ctx->hbstate, L.st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
    PR_HIP(hipStreamSynchronize(s));
    BatchState &hs = *ctx->hbstate;
    rc = stat_chunk(cs, ev, hs.head.phase_iter - before);
    if (rc != PR_OK) return rc;
    before = hs.head.phase_iter;
    for (int i = 0; i < Kc; ++i) master[orig[i]] = hs.col[i];
    if (hs.head.stop) break;
    if (rounds > max_iter + 2) {
      set_error("internal: update limit passed without stop");
      return PR_EDEVICE;
    }
    int act[kMaxCols], nact = 0;
    bool leaving[kMaxCols];
    for (int i = 0; i < Kc; ++i) {
      leaving[i] = !hs.col[i].active;
      if (hs.col[i].active) act[nact++] = i;
    }
    const int kp2 = batch_row_width(nact, fp32, narrow);
    if (ctx->compact == 0 || nact == Kc || kp2 >= kp) continue;
    // (a) columns leaving the layout: float32 -> their float64 columns (mixed), or final ranks
    if (mixed) {
      int map[kMaxCols];
      for (int i = 0; i < Kc; ++i) map[i] = leaving[i] ? orig[i] : -1;
      rc = write_cols(Kc, orig, map, false, nullptr);
      if (rc != PR_OK) return rc;
      PR_HIP(launch_batch_convert(s, (const float *)b0, (const float *)b1, kp, (float *)L.y64[1], (int32_t)N, Kc,
                                  L.st, L.cols));
    } else {
      rc = write_cols(Kc, orig, nullptr, true, leaving);
      if (rc != PR_OK) return rc;
      p.K = Kc;
      PR_HIP(launch_batch_output(s, false, outdeg, b0, b1, kp, (int32_t)N, Kc, p));
    }
    // (b) repack the active columns (all at the same parity) into the other buffer
    const int par = hs.col[act[0]].phase_updates & 1;
    void *cur = par ? b1 : b0, *oth = par ? b0 : b1;
    int norig[kMaxCols];
    for (int i = 0; i < nact; ++i) norig[i] = orig[act[i]];
    rc = write_cols(nact, norig, act, false, nullptr);
    if (rc != PR_OK) return rc;
    PR_HIP(launch_batch_compact(s, fp32, cur, kp, oth, kp2, (int32_t)N, nact, L.cols));
    // (c) the slot states follow their columns; the repacked buffer becomes buffer 0
    BatchState ns = hs;
    for (int i = 0; i < kMaxCols; ++i) {
      if (i < nact) {
        ns.col[i] = hs.col[act[i]];
        ns.col[i].phase_updates = 0;
      } else {
        memset(&ns.col[i], 0, sizeof ns.col[i]);
        ns.col[i].done = 1;
      }
    }
    hs = ns;
    PR_HIP(hipMemcpyAsync(L.st, &hs, sizeof(BatchState), hipMemcpyHostToDevice, s));
    PR_HIP(hipStreamSynchronize(s));
    Kc = nact;
    for (int i = 0; i < nact; ++i) orig[i] = norig[i];
    kp = kp2;
    b0 = oth;
    b1 = cur;
    p.K = Kc;
    p.grid = (int32_t)grid_of(fp32, kp);
    before = 0;
    hs.head.phase_iter = 0;
    PR_HIP(launch_fill_u32(s, (uint32_t *)&L.st->head.phase_iter, 1, 0u));
  }

  const BatchColumn *fin = master;
  if (mixed) {
    // remaining float32 columns -> float64, then the float64 phase over all K problems
    int map[kMaxCols];
    for (int i = 0; i < Kc; ++i) map[i] = orig[i];
    rc = write_cols(Kc, orig, map, false, nullptr);
    if (rc != PR_OK) return rc;
    PR_HIP(launch_batch_convert(s, (const float *)b0, (const float *)b1, kp, (float *)L.y64[1], (int32_t)N, Kc,
                                L.st, L.cols));
    // Every column is now in the column-major staging (the second float64 buffer, idle until the
    // float64 phase).  When every column goes on to the float64 phase, they are laid out as
    // float32 rows (the float32 buffers are free now) and the phase's first update reads those:
    // their float64 values are exact, so the update is the float64 one at half the bytes per
    // edge.  Otherwise (a column stopped by max_iter keeps its iterate in the float64 rows) as
    // float64 rows in the first buffer.
    bool live = true;
    for (int i = 0; i < K; ++i) live = live && !master[i].done;
    const bool rows32 = live && ctx->handover32 != 0;
    PR_HIP(launch_batch_rows(s, (const float *)L.y64[1], rows32 ? (void *)L.y32[0] : (void *)L.y64[0], !rows32, kp64,
                             (int32_t)N, K));
    int all[kMaxCols];
    for (int i = 0; i < K; ++i) all[i] = i;
    rc = write_cols(K, all, nullptr, true, nullptr);
    if (rc != PR_OK) return rc;
    BatchState &hs = *ctx->hbstate;
    memset(&hs, 0, sizeof hs);
    for (int i = 0; i < kMaxCols; ++i) {
      if (i < K) {
        hs.col[i] = master[i];
      } else {
        hs.col[i].done = 1;
      }
    }
    hs.phase = 2;
    PR_HIP(hipMemcpyAsync(L.st, &hs, sizeof(BatchState), hipMemcpyHostToDevice, s));
    PR_HIP(hipStreamSynchronize(s));
    PR_HIP(launch_batch_rearm(s, L.st, K));
    p.K = K;
    p.phase = 2;
    void *f0 = L.y64[0], *f1 = L.y64[1];
    bool stopped = false;
    if (rows32) {
      // the first float64 update: float32 rows in, float64 rows out to the second buffer, so that
      // every column's update parity (1) names that buffer and the later updates start from it
      BatchParams q = p;
      const int64_t res = ctx->max_grid > 0 ? ctx->max_grid : (int64_t)cus * batch_blocks_per_cu_f32rows(kp64);
      q.grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>({(int64_t)part.ndesc, res, kMaxGrid}));
      q.y_in = L.y32[0];
      q.y_out = L.y64[1];
      EventPair ev;
      if (ctx->timing) {
        PR_HIP(hipEventCreate(&ev.a));
        PR_HIP(hipEventCreate(&ev.b));
        PR_HIP(hipEventRecord(ev.a, s));
      }
      PR_HIP(launch_batch_update_f32rows(s, kp64, (unsigned)q.grid, q));
      if (ctx->timing) PR_HIP(hipEventRecord(ev.b, s));
      PR_HIP(hipMemcpyAsync(&ctx->hbstate->head, &L.st->head, sizeof(LoopHead), hipMemcpyDeviceToHost, s));
      PR_HIP(hipStreamSynchronize(s));
      stopped = ctx->hbstate->head.stop != 0;
      if (ctx->timing) {
        float ms = 0.f;
        PR_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        const ChunkSpec tag = batch_chunk(ctx, false, kp64, (unsigned)q.grid, q, nullptr, nullptr);
        ctx->stat_ms[tag.kind] += ms;
        ctx->stat_launches[tag.kind] += 1;
        ctx->stat_ms[tag.sub_kind] += ms;
        ctx->stat_launches[tag.sub_kind] += 1;
      }
      PR_HIP(launch_fill_u32(s, (uint32_t *)&L.st->head.phase_iter, 1, 0u));
      f0 = L.y64[1];
      f1 = L.y64[0];
    }
    p.grid = (int32_t)grid_of(false, kp64);
    int fbuf = 0;
    if (!stopped) {
      rc = run_until_stop(ctx, s, batch_chunk(ctx, false, kp64, (unsigned)p.grid, p, f0, f1), &L.st->head, max_iter,
                          &fbuf);
      if (rc != PR_OK) return rc;
    }
    PR_HIP(launch_batch_output(s, false, outdeg, L.y64[0], L.y64[1], kp64, (int32_t)N, K, p));
    PR_HIP(hipMemcpyAsync(ctx->hbstate, L.st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
    PR_HIP(hipStreamSynchronize(s));
    fin = ctx->hbstate->col;
  } else {
    rc = write_cols(Kc, orig, nullptr, true, nullptr);
    if (rc != PR_OK) return rc;
    p.K = Kc;
    PR_HIP(launch_batch_output(s, false, outdeg, b0, b1, kp, (int32_t)N, Kc, p));
    PR_HIP(hipStreamSynchronize(s));
  }
  int all_conv = 1;
  for (int k = 0; k < K; ++k) {
    const BatchColumn &c = fin[k];
    results[k].iterations = c.iters;
    results[k].converged = c.converged;
    results[k].fp32_iters = c.fp32_iters;
    results[k].fp64_iters = c.iters - c.fp32_iters;
    results[k].final_err[0] = c.err[0];
    results[k].final_err[1] = c.err[1];
    results[k].final_err[2] = c.err[2];
    all_conv &= c.converged;
  }
  return all_conv ? PR_OK : PR_NOT_CONVERGED;
}

// Workspace of pr_pull_sweep: the a = 1 iteration's state and partials, the column table, the
// iterates of one chunk (slot 0: the update's input, slots 1..kSweepChunk: its outputs), prep.
struct SweepLayout {
  SolveState *st;
  double *bpart;
  double *hpart;
  SweepCols *cols;
  FoldTable *fold;
  double *slots;
  int64_t stride;  // doubles between slots
  void *prep;
  size_t total;
};

static SweepLayout carve_sweep(void *ws, int64_t N, int64_t E, bool with_prep) {
  Carver c(ws);
  SweepLayout L{};
  L.st = (SolveState *)c.take(sizeof(SolveState));
  L.bpart = (double *)c.take(4 * sizeof(double) * (size_t)kMaxGrid);
  L.hpart = (double *)c.take(sizeof(double) * (size_t)max_slots(N, E));
  L.cols = (SweepCols *)c.take(sizeof(SweepCols));
  L.fold = (FoldTable *)c.take(sizeof(FoldTable));
  L.stride = (int64_t)(align_up(sizeof(double) * (size_t)N, 256) / sizeof(double));
  L.slots = (double *)c.take(sizeof(double) * (size_t)L.stride * (kSweepChunk + 1));
  L.prep = with_prep ? c.take(prep_bytes(N, E)) : nullptr;
  L.total = c.used;
  return L;
}

size_t pr_sweep_workspace_bytes(int64_t N, int64_t E, int32_t with_prep) {
  if (bad_graph_sizes(N, E)) return 0;
  return carve_sweep(nullptr, N, E, with_prep != 0).total;
}

int pr_pull_sweep(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                  const int32_t *outdeg, int64_t N, int64_t E, const void *prep, int32_t K, const pr_problem *probs,
                  double *const *ranks, double *const *norm_trace, void *workspace, size_t workspace_bytes,
                  pr_result *results) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !probs || !workspace || !results || (E > 0 && !in_indices)) {
    set_error("pr_pull_sweep: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  if (K < 1 || K > kMaxSweepCols) {
    set_error("K must be in [1, %d], got %d", kMaxSweepCols, K);
    return PR_EINVAL;
  }
  int max_iter = 1;
  for (int k = 0; k < K; ++k) {
    const pr_problem &q = probs[k];
    if (!(q.alpha >= 0.0 && q.alpha <= 1.0) || !(q.tau >= 0.0) || q.norm < PR_L1 || q.norm > PR_LINF ||
        q.max_iter < 1 || !ranks[k]) {
      set_error("problem %d: alpha in [0,1], tau >= 0, norm 1..3, max_iter >= 1 and a ranks buffer are required", k);
      return PR_EINVAL;
    }
    for (int k2 = 0; k2 < k; ++k2)
      if (ranks[k2] == ranks[k]) {
        set_error("problems %d and %d share a ranks buffer", k2, k);
        return PR_EINVAL;
      }
    max_iter = std::max(max_iter, q.max_iter);
  }
  const SweepLayout L = carve_sweep(workspace, N, E, prep == nullptr);
  if (workspace_bytes < L.total) {
    set_error("pr_pull_sweep: workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  int rc;
  const void *pp = prep;
  if (!prep) {
    rc = prepare_into(ctx, s, in_offsets, N, E, L.prep, &h);
    pp = L.prep;
  } else {
    rc = get_prep(ctx, s, prep, N, E, &h);
  }
  if (rc != PR_OK) return rc;

  // the column table (pinned staging, synchronised before the buffer is reused)
  SweepCols &hc = *ctx->hsweep;
  memset(&hc, 0, sizeof hc);
  hc.K = K;
  hc.remaining = K;
  for (int k = 0; k < K; ++k) {
    hc.alpha[k] = probs[k].alpha;
    hc.tau[k] = probs[k].tau;
    hc.norm[k] = probs[k].norm;
    hc.max_iter[k] = probs[k].max_iter;
    hc.ranks[k] = ranks[k];
    hc.trace[k] = norm_trace ? norm_trace[k] : nullptr;
  }
  PR_HIP(hipMemcpyAsync(L.cols, &hc, sizeof hc, hipMemcpyHostToDevice, s));
  // (the ranks need no clearing: the first fold writes every column)
  PR_HIP(launch_fill_u32(s, (uint32_t *)L.st, sizeof(SolveState) / 4, 0u));

  // the a = 1 iteration, as pr_pull's float64 solve (segmented when the prep has the layout)
  const std::pair<int32_t, int64_t> ts = tuned_settings(ctx, h);
  const int64_t gcap = ts.second > 0 ? ts.second : ctx->resident[0];
  const bool seg = ctx->segmented != 0 && h.seg_len > 0;
  const PrepPart &part = seg ? h.sl.merge_part : h.part[0];
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>({(int64_t)part.ndesc, gcap, kMaxGrid}));
  IterParams p{};
  p.off = in_offsets;
  p.idx = in_indices;
  if (seg) set_segmented(ctx, h, pp, false, p);
  p.outdeg = outdeg;
  p.desc = (const int4 *)((const char *)pp + part.desc_off);
  p.ndesc = part.ndesc;
  p.N = (int32_t)N;
  p.alpha = 1.0;
  p.tau = 0.0;
  p.norm = PR_L1;
  p.max_iter = max_iter;
  p.phase = 0;
  p.mid_deg = ts.first;
  p.st = L.st;
  p.bpart = L.bpart;
  p.hpart = L.hpart;
  p.hubs = (const int4 *)((const char *)pp + part.hub_off);
  p.nhubs = part.nhubs;
  p.grid = (int32_t)grid;
  p.trace = nullptr;
  p.sweep = L.cols;
  PR_HIP(launch_init(s, false, outdeg, (int32_t)N, nullptr, L.slots, 1.0, L.st, L.bpart, kMaxGrid));

  // chunk: update k reads slot k and writes slot k + 1
  ChunkSpec c;
  c.kind = PR_KERNEL_UPDATE_F64;
  c.count = kSweepChunk;
  {
    const int64_t meta[3] = {grid, kSweepChunk, (int64_t)(intptr_t)L.slots};
    c.key.resize(sizeof p + sizeof meta);
    memcpy(c.key.data(), &p, sizeof p);
    memcpy(c.key.data() + sizeof p, meta, sizeof meta);
  }
  const double *slots = L.slots;
  const int64_t stride = L.stride;
  c.launch = [grid, p, slots, stride](hipStream_t st, int k) {
    IterParams r = p;
    r.y_in = slots + (int64_t)k * stride;
    r.y_out = (void *)(slots + (int64_t)(k + 1) * stride);
    return launch_update(st, false, grid, r);
  };
  LoopHead *hh = (LoopHead *)ctx->hstate;
  int before = 0;
  bool first = true;
  EventPair fev;
  if (ctx->timing) {
    PR_HIP(hipEventCreate(&fev.a));
    PR_HIP(hipEventCreate(&fev.b));
  }
  for (int rounds = 0;; ++rounds) {
    const std::vector<hipEvent_t> *ev = nullptr;
    rc = run_chunk(ctx, s, c, &ev);
    if (rc != PR_OK) return rc;
    PR_HIP(hipMemcpyAsync(hh, &L.st->head, sizeof(LoopHead), hipMemcpyDeviceToHost, s));
    PR_HIP(hipStreamSynchronize(s));
    const int did = hh->phase_iter - before;
    if (ev && did > 0) {
      float ms = 0.f;
      for (int k = 0; k < did && k < c.count; ++k) {
        PR_HIP(hipEventElapsedTime(&ms, (*ev)[k], (*ev)[k + 1]));
        ctx->stat_ms[c.kind] += ms;
        ctx->stat_launches[c.kind] += 1;
      }
    }
    // fold the chunk's iterates (and the start, before the first update) into the columns
    const int32_t nfold = did + (first ? 1 : 0);
    if (nfold > 0) {
      if (ctx->timing) PR_HIP(hipEventRecord(fev.a, s));
      PR_HIP(launch_sweep_fold(s, L.slots, L.stride, first ? 0 : 1, nfold, first ? 0 : before + 1, outdeg,
                               (int32_t)N, L.cols, K, L.fold));
      if (ctx->timing) {
        PR_HIP(hipEventRecord(fev.b, s));
        PR_HIP(hipEventSynchronize(fev.b));
        float ms = 0.f;
        PR_HIP(hipEventElapsedTime(&ms, fev.a, fev.b));
        ctx->stat_ms[PR_KERNEL_SWEEP_FOLD] += ms;
        ctx->stat_launches[PR_KERNEL_SWEEP_FOLD] += 1;
      }
    }
    before = hh->phase_iter;
    first = false;
    if (hh->stop) break;
    if (rounds > max_iter) {  // cannot happen: the a = 1 iteration stops at max_iter
      set_error("internal: update limit passed without stop");
      return PR_EDEVICE;
    }
    // the chunk's last output becomes the next chunk's input
    PR_HIP(launch_copy_f64(s, L.slots + (int64_t)kSweepChunk * L.stride, L.slots, N));
  }
  PR_HIP(hipMemcpyAsync(&hc, L.cols, sizeof hc, hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  int all = 1;
  for (int k = 0; k < K; ++k) {
    results[k].iterations = hc.stop_iter[k];
    results[k].converged = hc.converged[k];
    results[k].fp32_iters = 0;
    results[k].fp64_iters = hc.stop_iter[k];
    results[k].final_err[0] = hc.err[k][0];
    results[k].final_err[1] = hc.err[k][1];
    results[k].final_err[2] = hc.err[k][2];
    all &= hc.converged[k];
  }
  return all ? PR_OK : PR_NOT_CONVERGED;
}

int pr_l1_distance(pr_ctx *ctx, void *stream, const double *x, const double *y, int64_t N, void *workspace,
                   size_t workspace_bytes, double *out) {
  if (!ctx || !x || !y || !workspace || !out) {
    set_error("pr_l1_distance: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1) {
    set_error("pr_l1_distance: N must be >= 1");
    return PR_EINVAL;
  }
  constexpr int32_t nb = 1024;
  if (workspace_bytes < (nb + 1) * sizeof(double)) {
    set_error("pr_l1_distance: workspace needs %zu bytes", (size_t)(nb + 1) * sizeof(double));
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  double *part = (double *)workspace;
  PR_HIP(launch_l1(s, x, y, N, part, nb));
  PR_HIP(hipMemcpyAsync(ctx->hscratch, part + nb, sizeof(double), hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  memcpy(out, ctx->hscratch, sizeof(double));
  return PR_OK;
}

}  // extern "C"
