// multi.hip -- many graphs, each with its own alpha / tau / norm / max_iter, solved in one
// persistent cooperative launch (paper, section 2 update and teleport term, section 3 error
// functions, applied to every graph of the batch).
//
// All graphs iterate in lockstep global rounds; a graph that stops stays untouched.  A round is
//   phase 1: every workgroup walks the global tile list (tile gi of graph g, in graph order, at
//            stride gridDim.x) with the single-vector tile code; row epilogues accumulate per
//            workgroup into the accumulator of the current graph, flushed to part[block][g]
//            whenever the graph changes; hub segment sums go to the graph's slot array;
//   grid barrier;
//   phase 2: graph g is finished by workgroup g % gridDim.x: hub rows (segments in order), the
//            partials of the workgroups that touched g in block order, then its teleport term,
//            errors, stop decision and trace row;
//   grid barrier; the loop ends when no graph is active.
// A grid barrier costs one release/acquire per workgroup (an L2 write-back/invalidate on gfx950),
// paid twice per round instead of once per tile.
#include <hip/hip_cooperative_groups.h>

#include "multi.h"

namespace cg = cooperative_groups;

namespace prpull {

__device__ __forceinline__ void flush_acc(const MultiParams &p, int g, Acc &a, double *red) {
  const double l1 = block_sum_n<kBlock>(a.l1, red);
  const double sq = block_sum_n<kBlock>(a.sq, red);
  const double mx = block_max_n<kBlock>(a.mx, red);
  const double dang = block_sum_n<kBlock>(a.dang, red);
  if (threadIdx.x == 0) {
    double *bp = p.part + ((int64_t)blockIdx.x * p.G + g) * 4;
    bp[0] = l1;
    bp[1] = sq;
    bp[2] = mx;
    bp[3] = dang;
  }
  a = Acc{0.0, 0.0, 0.0, 0.0};
}

// Graph owning global tile gi (binary search over the graphs' first tiles).
__device__ __forceinline__ int graph_of(const int32_t *__restrict__ base, int G, int32_t gi) {
  int lo = 0, hi = G - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= gi) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kBlock) void k_multi(MultiParams p) {
  __shared__ double vals[kSpan];
  __shared__ double red[kFinBlock / 64];
  __shared__ int s_any;
  cg::grid_group grid = cg::this_grid();
  const int t = threadIdx.x;
  for (int32_t round = 0; round < p.max_rounds; ++round) {
    // ---- phase 1: tiles of all active graphs
    int cur = -1;
    Acc a = {0.0, 0.0, 0.0, 0.0};
    TileCtx<double> c{};
    for (int32_t gi = blockIdx.x; gi < p.total_tiles; gi += gridDim.x) {
      const int g = graph_of(p.tile_base, p.G, gi);
      const MultiGraph &mg = p.graphs[g];
      MultiGraphState &gs = p.states[g];
      if (!gs.active) continue;
      if (g != cur) {
        if (cur >= 0) flush_acc(p, cur, a, red);
        cur = g;
        const int par = gs.iters & 1;
        c.off = mg.off;
        c.idx = mg.idx;
        c.outdeg = mg.outdeg;
        c.yin = mg.y[par];
        c.yout = mg.y[par ^ 1];
        c.hpart = mg.hpart;
        c.c0 = gs.c0;
        c.alpha = mg.alpha;
        c.mid_deg = mg.mid_deg;
      }
      const int32_t li = gi - p.tile_base[g];
      update_tile<double>(c, mg.desc[li], mg.desc[li + 1], a, vals, red);
    }
    if (cur >= 0) flush_acc(p, cur, a, red);
    grid.sync();

    // ---- phase 2: one workgroup per graph
    for (int g = blockIdx.x; g < p.G; g += gridDim.x) {
      const MultiGraph &mg = p.graphs[g];
      MultiGraphState &gs = p.states[g];
      if (!gs.active) continue;
      const int par = gs.iters & 1;
      const double *yin = mg.y[par];
      double *yout = mg.y[par ^ 1];
      Acc f = {0.0, 0.0, 0.0, 0.0};
      for (int32_t h = t; h < mg.nhubs; h += kBlock) {
        const int4 hb = mg.hubs[h];
        double s = 0.0;
#pragma unroll 1
        for (int32_t q = 0; q < hb.y; ++q) s += mg.hpart[hb.z + q];
        epilogue<double>(hb.x, s, gs.c0, mg.alpha, mg.outdeg[hb.x], yin[hb.x], yout, f);
      }
      // workgroups that walked a tile of g: tiles base .. base + ntiles - 1 at stride gridDim.x
      const int32_t base = p.tile_base[g], ntiles = p.tile_base[g + 1] - base;
      const int32_t nb = ntiles >= (int32_t)gridDim.x ? (int32_t)gridDim.x : ntiles;
      for (int32_t k = t; k < nb; k += kBlock) {
        const int32_t b = (base + k) % (int32_t)gridDim.x;
        const double *bp = p.part + ((int64_t)b * p.G + g) * 4;
        f.l1 += bp[0];
        f.sq += bp[1];
        f.mx = fmax(f.mx, bp[2]);
        f.dang += bp[3];
      }
      const double l1 = block_sum_n<kBlock>(f.l1, red);
      const double sq = block_sum_n<kBlock>(f.sq, red);
      const double mx = block_max_n<kBlock>(f.mx, red);
      const double dang = block_sum_n<kBlock>(f.dang, red);
      if (t == 0) {
#pragma clang fp contract(off)
        const double e[3] = {l1, sqrt(sq), mx};
        gs.err[0] = e[0];
        gs.err[1] = e[1];
        gs.err[2] = e[2];
        const int32_t it = gs.iters + 1;
        gs.iters = it;
        if (mg.trace) {
          mg.trace[3 * (int64_t)(it - 1) + 0] = e[0];
          mg.trace[3 * (int64_t)(it - 1) + 1] = e[1];
          mg.trace[3 * (int64_t)(it - 1) + 2] = e[2];
        }
        const double N = (double)mg.N;
        gs.c0 = (1.0 - mg.alpha) / N + (mg.alpha * dang) / N;
        const bool met = (mg.norm == 1 ? e[0] : mg.norm == 2 ? e[1] : e[2]) < mg.tau;
        if (met) {
          gs.converged = 1;
          gs.active = 0;
        } else if (it >= mg.max_iter) {
          gs.active = 0;
        }
      }
      __syncthreads();
    }
    grid.sync();
    if (t == 0) {
      int any = 0;
      for (int g = 0; g < p.G; ++g) any |= p.states[g].active;
      s_any = any;
    }
    __syncthreads();
    if (!s_any) break;
  }
}

// Start vectors (1/N or given) of every graph into its buffer 0, per-block dangling sums per graph.
__global__ __launch_bounds__(kBlock) void k_multi_init(MultiParams p) {
  __shared__ double red[kWaves];
  const int g = blockIdx.y;
  const MultiGraph &mg = p.graphs[g];
  double dang = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < mg.N; v += (int64_t)gridDim.x * kBlock) {
#pragma clang fp contract(off)
    const double r0 = mg.init ? mg.init[v] : 1.0 / (double)mg.N;
    const int32_t dv = mg.outdeg[v];
    if (dv > 0) {
      mg.y[0][v] = r0 / (double)dv;
    } else {
      mg.y[0][v] = r0;
      dang += r0;
    }
  }
  dang = block_sum(dang, red);
  if (threadIdx.x == 0) p.part[(int64_t)g * gridDim.x + blockIdx.x] = dang;
}

__global__ __launch_bounds__(kBlock) void k_multi_init_finish(MultiParams p, int32_t nb) {
  __shared__ double red[kWaves];
  const int g = blockIdx.x;
  const MultiGraph &mg = p.graphs[g];
  double D = 0.0;
  for (int32_t b = threadIdx.x; b < nb; b += kBlock) D += p.part[(int64_t)g * nb + b];
  D = block_sum(D, red);
  if (threadIdx.x == 0) {
#pragma clang fp contract(off)
    MultiGraphState &gs = p.states[g];
    const double N = (double)mg.N;
    gs.c0 = (1.0 - mg.alpha) / N + (mg.alpha * D) / N;
    gs.iters = 0;
    gs.active = 1;
    gs.converged = 0;
    gs.err[0] = gs.err[1] = gs.err[2] = 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_multi_output(MultiParams p) {
  const int g = blockIdx.y;
  const MultiGraph &mg = p.graphs[g];
  const double *y = mg.y[p.states[g].iters & 1];
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < mg.N; v += (int64_t)gridDim.x * kBlock) {
    const int32_t dv = mg.outdeg[v];
    mg.ranks[v] = dv > 0 ? y[v] * (double)dv : y[v];
  }
}

int multi_blocks_per_cu() {
  int n = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_multi, kBlock, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_multi(hipStream_t s, unsigned grid, const MultiParams &p, int32_t init_blocks) {
  hipLaunchKernelGGL(k_multi_init, dim3(init_blocks, p.G), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_multi_init_finish, dim3(p.G), dim3(kBlock), 0, s, p, init_blocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  MultiParams q = p;
  void *args[] = {&q};
  e = hipLaunchCooperativeKernel((const void *)k_multi, dim3(grid), dim3(kBlock), args, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_multi_output, dim3(init_blocks, p.G), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

}  // namespace prpull
