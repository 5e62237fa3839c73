// api_multi.hip -- the C ABI of the many-graph persistent launch (pr_pull_multi) and of the
// autotuner (pr_autotune).
#include <string.h>

#include <algorithm>

#include "api_internal.h"

extern "C" {

constexpr int32_t kMultiInitBlocks = 64;  // workgroups per graph of the start-vector kernels

// Update partial slots: graph g needs one per workgroup that owns one of its tiles, at most
// min(tiles, grid); bounded here by its largest possible tile count.
static int64_t multi_slot_bound(int32_t G, const pr_graph_problem *probs) {
  int64_t n = 0;
  for (int g = 0; g < G; ++g) n += std::min<int64_t>(max_desc(probs[g].N, probs[g].E, kTile, kRows), kMaxGrid);
  return n;
}

static size_t multi_layout(int32_t G, const pr_graph_problem *probs, void *ws, MultiGraph **graphs,
                           MultiGraphState **states, int32_t **tile_base, double **part, double **init_part,
                           GridBarrier **bar, double **hpart, double **y, void **preps) {
  Carver c(ws);
  *bar = (GridBarrier *)c.take(sizeof(GridBarrier));
  *graphs = (MultiGraph *)c.take(sizeof(MultiGraph) * (size_t)G);
  *states = (MultiGraphState *)c.take(sizeof(MultiGraphState) * (size_t)G);
  *tile_base = (int32_t *)c.take(sizeof(int32_t) * (size_t)(G + 1));
  *part = (double *)c.take(sizeof(double) * 4 * (size_t)multi_slot_bound(G, probs));
  *init_part = (double *)c.take(sizeof(double) * kMultiInitBlocks * (size_t)G);
  for (int g = 0; g < G; ++g) {
    hpart[g] = (double *)c.take(sizeof(double) * (size_t)max_slots(probs[g].N, probs[g].E));
    y[2 * g] = (double *)c.take(sizeof(double) * (size_t)probs[g].N);
    y[2 * g + 1] = (double *)c.take(sizeof(double) * (size_t)probs[g].N);
    preps[g] = probs[g].prep ? nullptr : c.take(prep_bytes(probs[g].N, probs[g].E));
  }
  return c.used;
}

size_t pr_multi_workspace_bytes(int32_t G, const pr_graph_problem *probs) {
  if (G < 1 || G > kMaxGraphs || !probs) return 0;
  for (int g = 0; g < G; ++g)
    if (bad_graph_sizes(probs[g].N, probs[g].E)) return 0;
  MultiGraph *a;
  MultiGraphState *b;
  int32_t *c;
  double *d, *d2;
  GridBarrier *e;
  std::vector<double *> hp(G), y(2 * G);
  std::vector<void *> pp(G);
  return multi_layout(G, probs, nullptr, &a, &b, &c, &d, &d2, &e, hp.data(), y.data(), pp.data());
}

int pr_pull_multi(pr_ctx *ctx, void *stream, int32_t G, const pr_graph_problem *probs, void *workspace,
                  size_t workspace_bytes, pr_result *results) {
  if (!ctx || !probs || !workspace || !results) {
    set_error("pr_pull_multi: NULL argument");
    return PR_EINVAL;
  }
  if (G < 1 || G > kMaxGraphs) {
    set_error("G must be in [1, %d], got %d", kMaxGraphs, G);
    return PR_EINVAL;
  }
  int max_rounds = 1;
  int64_t total_tiles = 0;
  for (int g = 0; g < G; ++g) {
    const pr_graph_problem &q = probs[g];
    if (!q.in_offsets || !q.outdeg || !q.ranks || (q.E > 0 && !q.in_indices)) {
      set_error("graph %d: NULL graph or ranks pointer", g);
      return PR_EINVAL;
    }
    if (bad_graph_sizes(q.N, q.E)) return PR_EINVAL;
    if (!(q.alpha >= 0.0 && q.alpha <= 1.0) || !(q.tau >= 0.0) || q.norm < PR_L1 || q.norm > PR_LINF ||
        q.max_iter < 1) {
      set_error("graph %d: alpha in [0,1], tau >= 0, norm 1..3 and max_iter >= 1 are required", g);
      return PR_EINVAL;
    }
    max_rounds = std::max(max_rounds, q.max_iter);
  }
  MultiGraph *dgraphs;
  MultiGraphState *dstates;
  int32_t *dbase;
  double *dpart, *dinit;
  GridBarrier *dbar;
  std::vector<double *> hpart(G), ybuf(2 * G);
  std::vector<void *> ownprep(G);
  const size_t need = multi_layout(G, probs, workspace, &dgraphs, &dstates, &dbase, &dpart, &dinit, &dbar,
                                   hpart.data(), ybuf.data(), ownprep.data());
  if (workspace_bytes < need) {
    set_error("pr_pull_multi: workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return PR_ENOMEM;
  }
  DeviceGuard dg(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  std::vector<MultiGraph> hg(G);
  std::vector<int32_t> base(G + 1, 0);
  for (int g = 0; g < G; ++g) {
    const pr_graph_problem &q = probs[g];
    PrepHeader h;
    int rc;
    const void *pp = q.prep;
    if (!pp) {
      rc = prepare_into(ctx, s, q.in_offsets, q.N, q.E, ownprep[g], &h);
      pp = ownprep[g];
    } else {
      rc = get_prep(ctx, s, pp, q.N, q.E, &h);
    }
    if (rc != PR_OK) return rc;
    const PrepPart &part = h.part[0];
    MultiGraph &m = hg[g];
    memset(&m, 0, sizeof m);
    m.off = q.in_offsets;
    m.idx = q.in_indices;
    m.outdeg = q.outdeg;
    m.desc = (const int4 *)((const char *)pp + part.desc_off);
    m.hubs = (const int4 *)((const char *)pp + part.hub_off);
    m.nhubs = part.nhubs;
    m.hpart = hpart[g];
    m.y[0] = ybuf[2 * g];
    m.y[1] = ybuf[2 * g + 1];
    m.init = q.init;
    m.ranks = q.ranks;
    m.trace = q.norm_trace;
    m.alpha = q.alpha;
    m.tau = q.tau;
    m.N = (int32_t)q.N;
    m.norm = q.norm;
    m.max_iter = q.max_iter;
    m.mid_deg = tuned_settings(ctx, h).first;
    total_tiles += part.ndesc;
    if (total_tiles > 2147483647LL) {
      set_error("pr_pull_multi: more than 2^31 tiles in one batch");
      return PR_EINVAL;
    }
    base[g + 1] = (int32_t)total_tiles;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1) cus = 1;
  const int64_t resident = (int64_t)cus * multi_blocks_per_cu();
  int64_t grid = ctx->max_grid > 0 ? std::min<int64_t>(ctx->max_grid, resident) : resident;
  grid = std::max<int64_t>(1, std::min<int64_t>({grid, total_tiles > 0 ? total_tiles : 1, (int64_t)kMaxGrid}));
  // partial slots: graph g's min(tiles, grid) workgroups, one slot each, graph after graph
  int64_t nslot = 0;
  for (int g = 0; g < G; ++g) {
    hg[g].pslot = (int32_t)nslot;
    nslot += std::min<int64_t>(base[g + 1] - base[g], grid);
  }
  if (nslot > multi_slot_bound(G, probs)) {
    set_error("internal: %lld partial slots exceed the workspace's %lld", (long long)nslot,
              (long long)multi_slot_bound(G, probs));
    return PR_EDEVICE;
  }
  // stage the tables through pinned memory (synchronised before the buffer is reused)
  const size_t tbytes = sizeof(MultiGraph) * (size_t)G + sizeof(int32_t) * (size_t)(G + 1);
  if (ctx->hmulti_bytes < tbytes) {
    if (ctx->hmulti) (void)hipHostFree(ctx->hmulti);
    ctx->hmulti = nullptr;
    ctx->hmulti_bytes = 0;
    PR_HIP(hipHostMalloc(&ctx->hmulti, tbytes, hipHostMallocDefault));
    ctx->hmulti_bytes = tbytes;
  }
  char *hm = (char *)ctx->hmulti;
  memcpy(hm, hg.data(), sizeof(MultiGraph) * (size_t)G);
  memcpy(hm + sizeof(MultiGraph) * (size_t)G, base.data(), sizeof(int32_t) * (size_t)(G + 1));
  PR_HIP(hipMemcpyAsync(dgraphs, hm, sizeof(MultiGraph) * (size_t)G, hipMemcpyHostToDevice, s));
  PR_HIP(hipMemcpyAsync(dbase, hm + sizeof(MultiGraph) * (size_t)G, sizeof(int32_t) * (size_t)(G + 1),
                        hipMemcpyHostToDevice, s));
  MultiParams p{};
  p.graphs = dgraphs;
  p.states = dstates;
  p.tile_base = dbase;
  p.part = dpart;
  p.init_part = dinit;
  p.bar = dbar;
  {
    int khz = 0;  // wall clock of the device (s_memrealtime), 100 MHz on this GPU family
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz < 1)
      khz = 100000;
    p.wait_ticks = (uint64_t)ctx->barrier_ms * (uint64_t)khz;
  }
  p.G = G;
  p.total_tiles = (int32_t)total_tiles;
  p.max_rounds = max_rounds;
  EventPair ev;  // destroyed on every return
  if (ctx->timing) {
    PR_HIP(hipEventCreate(&ev.a));
    PR_HIP(hipEventCreate(&ev.b));
    PR_HIP(hipEventRecord(ev.a, s));
  }
  PR_HIP(launch_fill_u32(s, (uint32_t *)dbar, sizeof(GridBarrier) / 4, 0u));
  PR_HIP(launch_multi(s, (unsigned)grid, p, kMultiInitBlocks));
  if (ctx->timing) PR_HIP(hipEventRecord(ev.b, s));
  std::vector<MultiGraphState> hs(G);
  uint32_t timed_out = 0;
  PR_HIP(hipMemcpyAsync(ctx->hmulti, dstates, sizeof(MultiGraphState) * (size_t)G, hipMemcpyDeviceToHost, s));
  PR_HIP(hipMemcpyAsync((char *)ctx->hmulti + sizeof(MultiGraphState) * (size_t)G, &dbar->timeout[0],
                        sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  memcpy(hs.data(), ctx->hmulti, sizeof(MultiGraphState) * (size_t)G);
  memcpy(&timed_out, (char *)ctx->hmulti + sizeof(MultiGraphState) * (size_t)G, sizeof(uint32_t));
  if (ctx->timing) {
    float ms = 0.f;
    PR_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    ctx->stat_ms[PR_KERNEL_MULTI] += ms;
    ctx->stat_launches[PR_KERNEL_MULTI] += 1;
  }
  if (timed_out) {
    set_error("pr_pull_multi: a grid barrier wait of the launch passed its time limit");
    return PR_EDEVICE;
  }
  int all = 1;
  for (int g = 0; g < G; ++g) {
    results[g].iterations = hs[g].iters;
    results[g].converged = hs[g].converged;
    results[g].fp32_iters = 0;
    results[g].fp64_iters = hs[g].iters;
    results[g].final_err[0] = hs[g].err[0];
    results[g].final_err[1] = hs[g].err[1];
    results[g].final_err[2] = hs[g].err[2];
    all &= hs[g].converged;
  }
  return all ? PR_OK : PR_NOT_CONVERGED;
}

// Workspace of pr_autotune: one region for the timed single and batch solves, then (prep == NULL)
// the tile partitions.
static size_t tune_region(int64_t N, int64_t E) {
  return std::max(carve(nullptr, N, E, PR_FP64, false).total,
                  carve_batch(nullptr, N, E, kTuneBatchCols, PR_MIXED, false).total);
}

size_t pr_tune_workspace_bytes(int64_t N, int64_t E, int32_t with_prep) {
  if (bad_graph_sizes(N, E)) return 0;
  return align_up(tune_region(N, E), 256) + (with_prep ? prep_bytes(N, E) : 0);
}

int pr_autotune(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                const int32_t *outdeg, int64_t N, int64_t E, void *prep, double *ranks, void *workspace,
                size_t workspace_bytes, pr_tune_result *out) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !workspace || !out || (E > 0 && !in_indices)) {
    set_error("pr_autotune: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  const size_t region = align_up(tune_region(N, E), 256);
  const size_t need = pr_tune_workspace_bytes(N, E, prep == nullptr);
  if (workspace_bytes < need) {
    set_error("pr_autotune: workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  void *pp = prep ? prep : (void *)((char *)workspace + region);
  PrepHeader h;
  int rc = prep ? get_prep(ctx, s, prep, N, E, &h) : prepare_into(ctx, s, in_offsets, N, E, pp, &h);
  if (rc != PR_OK) return rc;

  // saved settings; the candidates run with the autotuner's table off and explicit settings on
  const int64_t save_grid = ctx->max_grid, save_mid = ctx->mid_deg, save_timing = ctx->timing;
  const int64_t save_tuned = ctx->use_tuned, save_seg = ctx->segmented;
  const int64_t save_pair = ctx->pair_mid_deg, save_sgrid = ctx->seg_grid, save_mxcd = ctx->merge_xcd;
  const bool save_set = ctx->mid_deg_set, save_pair_set = ctx->pair_mid_deg_set,
             save_sgrid_set = ctx->seg_grid_set, save_mxcd_set = ctx->merge_xcd_set;
  int64_t save_launch[PR_KERNEL_KINDS];
  double save_ms[PR_KERNEL_KINDS];
  memcpy(save_launch, ctx->stat_launches, sizeof save_launch);
  memcpy(save_ms, ctx->stat_ms, sizeof save_ms);
  auto restore = [&]() {
    ctx->max_grid = save_grid;
    ctx->mid_deg = save_mid;
    ctx->mid_deg_set = save_set;
    ctx->timing = save_timing;
    ctx->use_tuned = save_tuned;
    ctx->segmented = save_seg;
    ctx->pair_mid_deg = save_pair;
    ctx->seg_grid = save_sgrid;
    ctx->merge_xcd = save_mxcd;
    ctx->pair_mid_deg_set = save_pair_set;
    ctx->seg_grid_set = save_sgrid_set;
    ctx->merge_xcd_set = save_mxcd_set;
    memcpy(ctx->stat_launches, save_launch, sizeof save_launch);
    memcpy(ctx->stat_ms, save_ms, sizeof save_ms);
  };
  ctx->timing = 1;
  ctx->segmented = 0;  // partition A's window and the thresholds are timed on the plain update
  auto mean_us = [&](int kind) {
    return ctx->stat_launches[kind] ? 1e3 * ctx->stat_ms[kind] / ctx->stat_launches[kind] : 1e300;
  };
  auto clear = [&](int kind) {
    ctx->stat_launches[kind] = 0;
    ctx->stat_ms[kind] = 0.0;
  };

  // ---- the single-vector update: partition A window x lane/wave threshold x grid
  const int tiles_a[] = {1024, 512, 256};
  const int32_t mids[] = {8, 16, 32, 64, 128};
  const int64_t res = ctx->resident[0];
  const int64_t grids[] = {res, 2 * res, 4 * res};
  const int tile_b0 = h.part[1].tile;
  double best = 1e300, dflt = 0.0;
  int best_tile = kTile;
  int32_t best_mid = kMidDeg, best_grid = (int32_t)std::min<int64_t>(res, kMaxGrid);
  int count = 0;
  constexpr int kReps = 4;
  ctx->use_tuned = 0;
  ctx->mid_deg_set = true;
  for (int ta : tiles_a) {
    rc = prepare_parts(ctx, s, in_offsets, N, E, pp, ta, tile_b0, &h, &h);
    if (rc != PR_OK) break;
    for (int64_t gsz : grids) {
      if (gsz > kMaxGrid) continue;
      for (int32_t m : mids) {
        ctx->max_grid = gsz;
        ctx->mid_deg = m;
        clear(PR_KERNEL_UPDATE_F64);
        pr_result r;
        rc = pr_pull(ctx, stream, in_offsets, in_indices, outdeg, N, E, pp, 0.85, 0.0, PR_L1, kReps, PR_FP64,
                     nullptr, ranks, nullptr, workspace, region, &r);
        if (rc < 0) break;
        const double us = mean_us(PR_KERNEL_UPDATE_F64);
        ++count;
        if (ta == kTile && gsz == res && m == kMidDeg) dflt = us;
        if (us < best) {
          best = us;
          best_tile = ta;
          best_mid = m;
          best_grid = (int32_t)gsz;
        }
      }
      if (rc < 0) break;
    }
    if (rc < 0) break;
  }
  // ---- the K-column float32 update: partition B window x threshold x workgroups per slot
  const int tiles_b[] = {256, 128};
  const int32_t mids_b[] = {16, 32, 64};
  const int32_t gmult[] = {1, 2};
  double best_b = 1e300, dflt_b = 0.0;
  int best_tile_b = kTileB;
  int32_t best_mid_b = kMidDeg, best_gm = 1;
  if (rc >= 0) {
    ctx->max_grid = 0;
    ctx->use_tuned = 1;  // the batch reads its candidate settings from the table
    pr_problem probs[kTuneBatchCols];
    double *rk[kTuneBatchCols];
    for (int k = 0; k < kTuneBatchCols; ++k) {
      probs[k] = pr_problem{0.85, 0.0, PR_L1, 3};
      rk[k] = ranks;  // outputs are not used; every column may write the same scratch
    }
    pr_result rb[kTuneBatchCols];
    for (int tb : tiles_b) {
      rc = prepare_parts(ctx, s, in_offsets, N, E, pp, best_tile, tb, &h, &h);
      if (rc != PR_OK) break;
      const std::vector<int64_t> sig = graph_signature(h);
      for (int32_t m : mids_b) {
        for (int32_t gm : gmult) {
          ctx->tuned_batch[sig] = {m, gm};
          clear(PR_KERNEL_BATCH_F32);
          rc = pr_pull_batch(ctx, stream, in_offsets, in_indices, outdeg, N, E, pp, kTuneBatchCols, probs, PR_MIXED,
                             nullptr, rk, nullptr, workspace, region, rb);
          if (rc < 0) break;
          const double us = mean_us(PR_KERNEL_BATCH_F32);
          ++count;
          if (tb == kTileB && m == kMidDeg && gm == 1) dflt_b = us;
          if (us < best_b) {
            best_b = us;
            best_tile_b = tb;
            best_mid_b = m;
            best_gm = gm;
          }
        }
        if (rc < 0) break;
      }
      ctx->tuned_batch.erase(sig);
      if (rc < 0) break;
    }
  }
  // ---- the source-segmented update, when the prep buffer holds that layout: pair threshold x
  // workgroups of the per-segment step x merge tile order (the merge on the single-vector
  // update's chosen threshold and grid, as it will run)
  const int32_t pmids[] = {64, 128, 256, 512};
  const int64_t sgrids[] = {res, 2 * res};
  SegTune best_st{kPairMidDeg, 0, 0};
  double best_s = 0.0, dflt_s = 0.0;
  int count_s = 0;
  if (rc >= 0 && h.seg_len > 0) {
    best_s = 1e300;
    ctx->segmented = 1;
    ctx->use_tuned = 0;
    ctx->max_grid = best_grid;
    ctx->mid_deg = best_mid;
    ctx->mid_deg_set = true;
    ctx->pair_mid_deg_set = ctx->seg_grid_set = ctx->merge_xcd_set = true;
    for (int32_t pm : pmids) {
      for (int64_t sg : sgrids) {
        if (sg > kMaxGrid) continue;
        for (int mx = 0; mx < 2; ++mx) {
          ctx->pair_mid_deg = pm;
          ctx->seg_grid = sg;
          ctx->merge_xcd = mx;
          clear(PR_KERNEL_UPDATE_F64);
          pr_result r;
          rc = pr_pull(ctx, stream, in_offsets, in_indices, outdeg, N, E, pp, 0.85, 0.0, PR_L1, kReps, PR_FP64,
                       nullptr, ranks, nullptr, workspace, region, &r);
          if (rc < 0) break;
          const double us = mean_us(PR_KERNEL_UPDATE_F64);
          ++count_s;
          if (pm == kPairMidDeg && sg == res && mx == 0) dflt_s = us;
          if (us < best_s) {
            best_s = us;
            best_st = SegTune{pm, (int32_t)sg, mx};
          }
        }
        if (rc < 0) break;
      }
      if (rc < 0) break;
    }
  }
  restore();
  if (rc < 0) return rc;
  // the chosen windows stay in the prep buffer; the thresholds and grids go to the table
  rc = prepare_parts(ctx, s, in_offsets, N, E, pp, best_tile, best_tile_b, &h, &h);
  if (rc != PR_OK) return rc;
  if (h.seg_len > 0) {
    const std::vector<int64_t> ssig = seg_signature(h);
    ctx->tuned_seg[ssig] = best_st;
    save_tune_seg_entry(ctx, ssig, best_st);
  }
  const std::vector<int64_t> sig = graph_signature(h);
  ctx->tuned[sig] = {best_mid, best_grid};
  ctx->tuned_batch[sig] = {best_mid_b, best_gm};
  save_tune_entry(ctx, sig, best_mid, best_grid, best_mid_b, best_gm);
  out->mid_deg = best_mid;
  out->grid = best_grid;
  out->tile = best_tile;
  out->rows = best_tile / 2;
  out->mid_deg_batch = best_mid_b;
  out->grid_batch_factor = best_gm;
  out->tile_batch = best_tile_b;
  out->rows_batch = best_tile_b / 2;
  out->candidates = count;
  out->pad = 0;
  out->best_us = best;
  out->default_us = dflt;
  out->best_batch_us = best_b;
  out->default_batch_us = dflt_b;
  out->pair_mid_deg = h.seg_len > 0 ? best_st.pair_mid_deg : 0;
  out->seg_grid = h.seg_len > 0 ? best_st.seg_grid : 0;
  out->merge_xcd = h.seg_len > 0 ? best_st.merge_xcd : 0;
  out->seg_candidates = count_s;
  out->best_seg_us = best_s;
  out->default_seg_us = dflt_s;
  return PR_OK;
}

}  // extern "C"
