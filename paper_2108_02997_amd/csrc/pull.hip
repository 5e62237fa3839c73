// pull.hip -- the per-update kernels of the pull PageRank (paper, section 2 update and
// teleport term; section 3 error functions).
//
// State layout.  One vector y[N] per iterate, in the arithmetic type VT of the phase:
//   y_u = r_u / d_u  for a vertex with out-edges (its contribution to every out-neighbour),
//   y_u = r_u        for a dangling vertex (never gathered: it has no out-edges).
// The gather reads y directly, so the contribution pass r/d is fused into the previous
// update's epilogue and no separate contribution array exists.  The previous rank of a
// vertex is recovered as y_u * d_u: exact for float32 y (the product of a 24-bit significand
// and d < 2^29 fits in float64), within one float64 rounding for float64 y.
//
// One update = one launch of k_update over all tiles (see prep.hip), with
//   gather   : contributions of a tile's in-edges staged through LDS (coalesced index loads);
//   sum      : one lane per low in-degree row, one wave64 per mid row, one workgroup per
//              segment of a long row (fixed-order block reduction);
//   epilogue : r'_v = c0 + alpha*s_v, the new y_v, |r'_v - r_v| into L1/L2/Linf partials and
//              r'_v of dangling vertices into the dangling-sum partial;
// then k_finish (one block, after the kernel boundary) combines hub segments in segment order,
// reduces the block partials in block order and sets the errors, the next teleport term
// c0 = (1-alpha)/N + (alpha*D)/N, the stop flags and the trace row.
// Every reduction has a fixed order, so results are bitwise repeatable run to run.
#include "device.h"

namespace prpull {

// Finalize one update (lane 0 of the finishing kernel), with the reduced totals.
__device__ __forceinline__ void finalize(const IterParams &p, double l1, double sq, double mx, double dang) {
#pragma clang fp contract(off)
  SolveState *st = p.st;
  const double e[3] = {l1, sqrt(sq), mx};
  st->err[0] = e[0];
  st->err[1] = e[1];
  st->err[2] = e[2];
  const int32_t it = st->head.iter + 1;
  st->head.iter = it;
  st->head.phase_iter = st->head.phase_iter + 1;
  if (p.trace) {
    p.trace[3 * (int64_t)(it - 1) + 0] = e[0];
    p.trace[3 * (int64_t)(it - 1) + 1] = e[1];
    p.trace[3 * (int64_t)(it - 1) + 2] = e[2];
  }
  const double N = (double)p.N;
  st->c0 = (1.0 - p.alpha) / N + (p.alpha * dang) / N;
  if (p.sweep) {
    // the a = 1 iteration of a sweep: column k's change at this update is alpha_k^it times this
    // update's change, in every norm; a column stops at the first update where that meets its
    // tau in its norm, or at its max_iter
    SweepCols *sw = p.sweep;
    int32_t rem = 0;
    for (int k = 0; k < sw->K; ++k) {
      if (sw->stop_iter[k]) continue;
      const double ak = pow(sw->alpha[k], (double)it);
      const double ek[3] = {ak * e[0], ak * e[1], ak * e[2]};
      sw->err[k][0] = ek[0];
      sw->err[k][1] = ek[1];
      sw->err[k][2] = ek[2];
      if (sw->trace[k]) {
        sw->trace[k][3 * (int64_t)(it - 1) + 0] = ek[0];
        sw->trace[k][3 * (int64_t)(it - 1) + 1] = ek[1];
        sw->trace[k][3 * (int64_t)(it - 1) + 2] = ek[2];
      }
      const int nk = sw->norm[k];
      if ((nk == 1 ? ek[0] : nk == 2 ? ek[1] : ek[2]) < sw->tau[k]) {
        sw->converged[k] = 1;
        sw->stop_iter[k] = it;
      } else if (it >= sw->max_iter[k]) {
        sw->stop_iter[k] = it;
      } else {
        ++rem;
      }
    }
    sw->remaining = rem;
    if (rem == 0 || it >= p.max_iter) {
      st->head.stop = 1;
      st->head.done = 1;
    }
    return;
  }
  if (p.snap) {
    // rank snapshots (single-phase solves): the same test as the solve's own stop below
    SnapTable *sn = p.snap;
    unsigned long long m = 0;
    for (int i = 0; i < sn->S; ++i) {
      if (sn->iter[i]) continue;
      const int ni = sn->norm[i];
      if ((ni == 1 ? e[0] : ni == 2 ? e[1] : e[2]) < sn->tau[i]) {
        sn->iter[i] = it;
        m |= 1ull << i;
      }
    }
    sn->pending = m;
    sn->src = p.y_out;
    sn->node = p.node;
  }
  const bool met = (p.norm == 1 ? e[0] : p.norm == 2 ? e[1] : e[2]) < p.tau;
  if (p.phase == 1) {
    // float32 phase: hand over to float64 once tau is met, the L1 change stops shrinking (in
    // exact arithmetic it never grows: the update is an alpha-contraction in L1) or, for the L1
    // norm, the change is below kL1Handover
    if (met) st->met32 = 1;
    if (met || !(l1 < st->prev_l1) || (p.norm == 1 && l1 < kL1Handover)) st->head.stop = 1;
    st->prev_l1 = l1;
    if (it >= p.max_iter) {
      st->head.stop = 1;
      st->head.done = 1;
    }
  } else {
    if (met) {
      st->converged = 1;
      st->head.stop = 1;
      st->head.done = 1;
    } else if (it >= p.max_iter) {
      st->head.stop = 1;
      st->head.done = 1;
    }
  }
}

// ------------------------------------------------------------------ the update kernel
// Blocks take tiles i = blockIdx.x, blockIdx.x + grid, ... and write their four partial sums
// with plain stores; all cross-block combining happens in k_finish, after the kernel boundary
// (device-scope fences would write back and invalidate the whole L2 of each XCD).
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_update(IterParams p) {
  __shared__ VT vals[kSpan];
  __shared__ double red[kWaves];
  const SolveState *st = p.st;
  if (st->head.stop) return;
  TileCtx<VT> c;
  c.off = p.off;
  c.idx = p.idx;
  c.outdeg = p.outdeg;
  c.yin = (const VT *)p.y_in;
  c.xs = p.partial ? (const VT *)p.partial : c.yin;
  c.yout = (VT *)p.y_out;
  c.hpart = p.hpart;
  c.c0 = st->c0;
  c.alpha = p.alpha;
  c.mid_deg = p.mid_deg;
  const int t = threadIdx.x;
  Acc a = {0.0, 0.0, 0.0, 0.0};
  if (p.partial && p.merge_xcd && (gridDim.x & 7) == 0) {
    // merge step: workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD b % 8),
    // so XCD x takes the x-th eighth of the tiles; neighbouring tiles read neighbouring partial
    // sums of every segment, which then share lines in that XCD's L2
    const int32_t x = blockIdx.x & 7, nx = gridDim.x >> 3;
    const int32_t lo = (int32_t)((int64_t)p.ndesc * x / 8), hi = (int32_t)((int64_t)p.ndesc * (x + 1) / 8);
    for (int32_t i = lo + (int32_t)(blockIdx.x >> 3); i < hi; i += nx)
      update_tile<VT>(c, p.desc[i], p.desc[i + 1], a, vals, red);
  } else {
    for (int32_t i = blockIdx.x; i < p.ndesc; i += gridDim.x)
      update_tile<VT>(c, p.desc[i], p.desc[i + 1], a, vals, red);
  }

  const double l1 = block_sum_n<kBlock>(a.l1, red);
  const double sq = block_sum_n<kBlock>(a.sq, red);
  const double mx = block_max_n<kBlock>(a.mx, red);
  const double dang = block_sum_n<kBlock>(a.dang, red);
  if (t == 0) {
    double *bp = p.bpart + 4 * (int64_t)blockIdx.x;
    bp[0] = l1;
    bp[1] = sq;
    bp[2] = mx;
    bp[3] = dang;
  }
}

// Per-segment step of the source-segmented update: every pair's entries of the iterate summed
// into its partial (pairs listed segment by segment, so the workgroups running at one time
// gather from one or two segments' slice of the iterate, which the XCDs' L2 caches hold).
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_seg_gather(IterParams p) {
  __shared__ VT vals[kSpan];
  __shared__ double red[kWaves];
  if (p.st->head.stop) return;
  TileCtx<VT> c{};
  c.off = p.poff;
  c.idx = p.sidx;
  c.xs = (const VT *)p.y_in;
  c.part = (VT *)p.partial;
  c.mid_deg = p.pair_mid_deg;
  Acc a = {0.0, 0.0, 0.0, 0.0};
  if (p.seg_xcd && (gridDim.x & 7) == 0) {
    // workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD b % 8), so XCD x
    // takes the x-th eighth of the tiles: each XCD walks a few segments of its own, and every
    // segment's slice of the iterate is fetched into one XCD's L2 instead of all eight
    const int32_t x = blockIdx.x & 7, nx = gridDim.x >> 3;
    const int32_t lo = (int32_t)((int64_t)p.npdesc * x / 8), hi = (int32_t)((int64_t)p.npdesc * (x + 1) / 8);
    for (int32_t i = lo + (int32_t)(blockIdx.x >> 3); i < hi; i += nx)
      update_tile<VT, true>(c, p.pdesc[i], p.pdesc[i + 1], a, vals, red);
  } else {
    for (int32_t i = blockIdx.x; i < p.npdesc; i += gridDim.x)
      update_tile<VT, true>(c, p.pdesc[i], p.pdesc[i + 1], a, vals, red);
  }
}

// One block: hub rows (segment partials combined in segment order, then the epilogue), the
// update kernel's block partials in block order, and the finalize.
template <typename VT>
__global__ __launch_bounds__(kFinBlock) void k_finish(IterParams p) {
  __shared__ double red[kFinBlock / 64];
  SolveState *st = p.st;
  if (st->head.stop) return;
  const double c0 = st->c0;
  const VT *__restrict__ yin = (const VT *)p.y_in;
  VT *__restrict__ yout = (VT *)p.y_out;
  Acc a = {0.0, 0.0, 0.0, 0.0};
  for (int32_t h = threadIdx.x; h < p.nhubs; h += kFinBlock) {
    const int4 hb = p.hubs[h];
    double s = 0.0;
    for (int32_t q = 0; q < hb.y; ++q) s += p.hpart[hb.z + q];
    epilogue<VT>(hb.x, s, c0, p.alpha, p.outdeg[hb.x], yin[hb.x], yout, a);
  }
  for (int32_t b = threadIdx.x; b < p.grid; b += kFinBlock) {
    const double *bp = p.bpart + 4 * (int64_t)b;
    a.l1 += bp[0];
    a.sq += bp[1];
    a.mx = fmax(a.mx, bp[2]);
    a.dang += bp[3];
  }
  const double l1 = block_sum_n<kFinBlock>(a.l1, red);
  const double sq = block_sum_n<kFinBlock>(a.sq, red);
  const double mx = block_max_n<kFinBlock>(a.mx, red);
  const double dang = block_sum_n<kFinBlock>(a.dang, red);
  if (threadIdx.x == 0) finalize(p, l1, sq, mx, dang);
}

// ------------------------------------------------------------------ init, convert, output
// y0 from the start vector (or 1/N); per-block dangling sums of the start vector.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_init(const int32_t *__restrict__ outdeg, int32_t N,
                                                 const double *__restrict__ init, VT *__restrict__ y,
                                                 double *bpart) {
#pragma clang fp contract(off)
  __shared__ double red[kWaves];
  double dang = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock) {
    const double r0 = init ? init[v] : 1.0 / (double)N;
    const int32_t dv = outdeg[v];
    if (dv > 0) {
      y[v] = (VT)(r0 / (double)dv);
    } else {
      const VT yy = (VT)r0;
      y[v] = yy;
      dang += (double)yy;
    }
  }
  dang = block_sum(dang, red);
  if (threadIdx.x == 0) bpart[blockIdx.x] = dang;
}

// One block: c0 of the first update from the start vector's dangling sum; resets the state.
__global__ __launch_bounds__(kFinBlock) void k_init_finish(const double *__restrict__ bpart, int32_t nb, int32_t N,
                                                           double alpha, SolveState *st) {
#pragma clang fp contract(off)
  __shared__ double red[kFinBlock / 64];
  double D = 0.0;
  for (int32_t b = threadIdx.x; b < nb; b += kFinBlock) D += bpart[b];
  D = block_sum_n<kFinBlock>(D, red);
  if (threadIdx.x == 0) {
    const double Nd = (double)N;
    st->c0 = (1.0 - alpha) / Nd + (alpha * D) / Nd;
    st->head.iter = 0;
    st->head.phase_iter = 0;
    st->head.stop = 0;
    st->head.done = 0;
    st->converged = 0;
    st->met32 = 0;
    st->prev_l1 = __builtin_huge_val();
  }
}

// Float32 iterate -> float64 iterate (same implied ranks).
__global__ __launch_bounds__(kBlock) void k_convert(const float *__restrict__ y32, double *__restrict__ y64,
                                                    int32_t N) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock)
    y64[v] = (double)y32[v];
}

// Re-arm the update kernels for the float64 phase (after k_convert, kernel-ordered).
__global__ void k_rearm(SolveState *st) {
  if (threadIdx.x == 0) {
    st->head.stop = st->head.done;
    st->head.phase_iter = 0;
  }
}

// ranks_v = y_v * d_v (or y_v for a dangling vertex).
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_output(const int32_t *__restrict__ outdeg, const VT *__restrict__ y,
                                                   int32_t N, double *__restrict__ ranks) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock) {
    const int32_t dv = outdeg[v];
    ranks[v] = dv > 0 ? (double)y[v] * (double)dv : (double)y[v];
  }
}

// The rank snapshots the update at chunk position p.node took (finalize): ranks_v as k_output
// writes them, into every such snapshot.  Runs after every update of a solve with snapshots and
// copies only after the update that took some (a chunk's updates after the stop do not run
// finalize, so a later position never matches).
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_snap(IterParams p) {
  const SnapTable *sn = p.snap;
  const unsigned long long m = sn->pending;
  if (m == 0 || sn->node != p.node) return;
  const VT *__restrict__ y = (const VT *)sn->src;
  double *__restrict__ out = sn->out;
  const int64_t N = p.N;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock) {
    const int32_t dv = p.outdeg[v];
    const double r = dv > 0 ? (double)y[v] * (double)dv : (double)y[v];
    for (unsigned long long b = m; b; b &= b - 1) out[(int64_t)(__ffsll((long long)b) - 1) * N + v] = r;
  }
}

// Sum of |x_v - y_v|: per-block partials, then one block in block order.
__global__ __launch_bounds__(kBlock) void k_l1_partial(const double *__restrict__ x, const double *__restrict__ y,
                                                       int64_t N, double *__restrict__ part) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock)
    s += fabs(x[v] - y[v]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kFinBlock) void k_l1_final(double *part, int32_t nb) {
  __shared__ double red[kFinBlock / 64];
  double s = 0.0;
#pragma unroll 1
  for (int32_t b = threadIdx.x; b < nb; b += kFinBlock) s += part[b];
  s = block_sum_n<kFinBlock>(s, red);
  if (threadIdx.x == 0) part[nb] = s;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_l1(hipStream_t s, const double *x, const double *y, int64_t N, double *part, int32_t nb) {
  hipLaunchKernelGGL(k_l1_partial, dim3(nb), dim3(kBlock), 0, s, x, y, N, part);
  hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kFinBlock), 0, s, part, nb);
  return hipGetLastError();
}

static unsigned grid_for(int64_t n, int64_t cap) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_init(hipStream_t s, bool fp32, const int32_t *outdeg, int32_t N, const double *init, void *y,
                       double alpha, SolveState *st, double *bpart, int64_t bpart_cap) {
  const unsigned g = grid_for(N, bpart_cap < 1024 ? bpart_cap : 1024);
  if (fp32)
    hipLaunchKernelGGL(k_init<float>, dim3(g), dim3(kBlock), 0, s, outdeg, N, init, (float *)y, bpart);
  else
    hipLaunchKernelGGL(k_init<double>, dim3(g), dim3(kBlock), 0, s, outdeg, N, init, (double *)y, bpart);
  hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(kFinBlock), 0, s, (const double *)bpart, (int32_t)g, N, alpha, st);
  return hipGetLastError();
}

// Resident workgroups of the update kernel per compute unit.
int update_blocks_per_cu(bool fp32) {
  int n = 0;
  hipError_t e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_update<float>, kBlock, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_update<double>, kBlock, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

// One update = the tile kernel and the one-block finishing kernel (source-segmented: the
// per-segment step, then the merge step as the tile kernel, then the finishing kernel).
hipError_t launch_update(hipStream_t s, bool fp32, unsigned grid, const IterParams &p) {
  if (p.poff) {
    if (fp32)
      hipLaunchKernelGGL(k_seg_gather<float>, dim3((unsigned)p.pgrid), dim3(kBlock), 0, s, p);
    else
      hipLaunchKernelGGL(k_seg_gather<double>, dim3((unsigned)p.pgrid), dim3(kBlock), 0, s, p);
  }
  if (fp32) {
    hipLaunchKernelGGL(k_update<float>, dim3(grid), dim3(kBlock), 0, s, p);
    hipLaunchKernelGGL(k_finish<float>, dim3(1), dim3(kFinBlock), 0, s, p);
  } else {
    hipLaunchKernelGGL(k_update<double>, dim3(grid), dim3(kBlock), 0, s, p);
    hipLaunchKernelGGL(k_finish<double>, dim3(1), dim3(kFinBlock), 0, s, p);
  }
  return hipGetLastError();
}

hipError_t launch_convert(hipStream_t s, const float *y32, double *y64, int32_t N, SolveState *st) {
  hipLaunchKernelGGL(k_convert, dim3(grid_for(N, 2048)), dim3(kBlock), 0, s, y32, y64, N);
  hipLaunchKernelGGL(k_rearm, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_snap(hipStream_t s, bool fp32, const IterParams &p) {
  if (fp32)
    hipLaunchKernelGGL(k_snap<float>, dim3(grid_for(p.N, 2048)), dim3(kBlock), 0, s, p);
  else
    hipLaunchKernelGGL(k_snap<double>, dim3(grid_for(p.N, 2048)), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_output(hipStream_t s, bool fp32, const int32_t *outdeg, const void *y, int32_t N, double *ranks) {
  if (fp32)
    hipLaunchKernelGGL(k_output<float>, dim3(grid_for(N, 2048)), dim3(kBlock), 0, s, outdeg, (const float *)y, N,
                       ranks);
  else
    hipLaunchKernelGGL(k_output<double>, dim3(grid_for(N, 2048)), dim3(kBlock), 0, s, outdeg, (const double *)y,
                       N, ranks);
  return hipGetLastError();
}

}  // namespace prpull
