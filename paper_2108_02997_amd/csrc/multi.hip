// multi.hip -- many graphs, each with its own alpha / tau / norm / max_iter, solved in one
// persistent cooperative launch (paper, section 2 update and teleport term, section 3 error
// functions, applied to every graph of the batch).
//
// All graphs iterate in lockstep global rounds; a graph that stops stays untouched.  A round is
//   phase 1: the graphs' tiles are numbered globally in graph order and global tile gi belongs
//            to workgroup gi % gridDim.x; every workgroup takes, graph by graph, its tiles of the
//            active graphs with the single-vector tile code; row epilogues accumulate per
//            workgroup and graph and are flushed to part[block][g]; hub segment sums go to the
//            graph's slot array;
//   grid barrier;
//   phase 2: graph g is finished by workgroup g % gridDim.x: hub rows (segments in order), the
//            partials of the workgroups that touched g in block order, then its teleport term,
//            errors, stop decision and trace row;
//   grid barrier; the loop ends when no graph is active.
//
// Grid barrier.  A device-scope release is a write-back of the XCD's whole L2 on gfx950 and an
// acquire an invalidate of it (and of the CU's L1); issued by every workgroup, as a generic grid
// barrier does, they cost ~220 us per barrier at 2048 workgroups.  Here the release is paid once
// per XCD: every lane waits until its stores have reached the XCD's L2, the last workgroup of
// the XCD to arrive (per-XCD arrival count) writes that L2 back for all of them and arrives at
// the global count; once every XCD has arrived it invalidates its L2 and releases the XCD's
// workgroups, which each acquire (invalidate) before reading.  ~21 us at 2048 workgroups.  Every
// wait has a time limit: past it the workgroup sets `timeout` and leaves, so does every other
// one at its next wait, and the host reports the failure.  The limit is the context's
// "barrier_ms" (5 s by default).
#include "multi.h"

namespace prpull {

__device__ __forceinline__ uint32_t xcc_id() {
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & (kMaxXcd - 1);
}

__device__ __forceinline__ uint32_t bar_load(uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t bar_add(uint32_t *p) {
  return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p >= target; false after `limit` wall-clock ticks or once another workgroup has
// timed out.
__device__ bool bar_wait(GridBarrier *b, uint32_t *p, uint32_t target, uint64_t limit) {
  const uint64_t t0 = wall_clock64();
  while (bar_load(p) < target) {
    if (bar_load(&b->timeout[0]) || wall_clock64() - t0 > limit) {
      __hip_atomic_store(&b->timeout[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

struct BarSlot {
  uint32_t x;     // this workgroup's XCD
  uint32_t nx;    // workgroups on it
  uint32_t nxcd;  // XCDs with workgroups of the launch
};

// Count the launch's workgroups per XCD.  Every workgroup adds itself to its XCD's count and
// then waits until the per-XCD counts sum to the grid: the words it waits on are the counted
// words themselves, and since each only grows, a total of gridDim.x means every count is final
// (no ordering between atomics on different words is relied on).  Block-uniform result; false
// on time-out.
__device__ bool bar_setup(GridBarrier *b, BarSlot &slot, uint64_t limit) {
  __shared__ uint32_t s_v[3];
  int ok = 1;
  if (threadIdx.x == 0) {
    const uint32_t x = xcc_id();
    bar_add(&b->members[x * kBarPad]);
    const uint64_t t0 = wall_clock64();
    uint32_t n = 0;
    for (;;) {
      uint32_t total = 0;
      n = 0;
      for (int i = 0; i < kMaxXcd; ++i) {
        const uint32_t c = bar_load(&b->members[i * kBarPad]);
        total += c;
        n += c > 0;
      }
      if (total >= gridDim.x) break;
      if (bar_load(&b->timeout[0]) || wall_clock64() - t0 > limit) {
        __hip_atomic_store(&b->timeout[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    s_v[0] = x;
    s_v[1] = bar_load(&b->members[x * kBarPad]);  // final once the counts sum to the grid
    s_v[2] = n;
  }
  if (__syncthreads_or(!ok)) return false;
  slot = BarSlot{s_v[0], s_v[1], s_v[2]};
  return true;
}

// Barrier number k (1, 2, ...) of the launch.  Block-uniform result; false on time-out.
__device__ bool grid_barrier(GridBarrier *b, const BarSlot &slot, uint32_t k, uint64_t limit) {
  __builtin_amdgcn_s_waitcnt(0);  // this lane's stores are in the XCD's L2
  __syncthreads();
  int ok = 1;
  if (threadIdx.x == 0) {
    if (bar_add(&b->xcd[slot.x * kBarPad]) + 1u == k * slot.nx) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the XCD's L2 to memory
      bar_add(&b->global[0]);
      ok = bar_wait(b, &b->global[0], k * slot.nxcd, limit);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&b->release[slot.x * kBarPad], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      ok = bar_wait(b, &b->release[slot.x * kBarPad], k, limit);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __builtin_amdgcn_s_waitcnt(0);
  }
  return !__syncthreads_or(!ok);
}

// The workgroup's partials of graph g into its slot k (its rank among the workgroups that own a
// tile of g: k = first tile - the graph's first tile).
__device__ __forceinline__ void flush_acc(const MultiParams &p, int64_t slot, Acc &a, double *red) {
  const double l1 = block_sum_n<kBlock>(a.l1, red);
  const double sq = block_sum_n<kBlock>(a.sq, red);
  const double mx = block_max_n<kBlock>(a.mx, red);
  const double dang = block_sum_n<kBlock>(a.dang, red);
  if (threadIdx.x == 0) {
    double *bp = p.part + slot * 4;
    bp[0] = l1;
    bp[1] = sq;
    bp[2] = mx;
    bp[3] = dang;
  }
  a = Acc{0.0, 0.0, 0.0, 0.0};
}

__global__ __launch_bounds__(kBlock) void k_multi(MultiParams p) {
  __shared__ double vals[kSpan];
  __shared__ double red[kFinBlock / 64];
  __shared__ int32_t s_act[kBlock], s_base[kBlock + 1];
  const int t = threadIdx.x;
  const int32_t nblk = (int32_t)gridDim.x, blk = (int32_t)blockIdx.x;
  BarSlot slot;
  if (!bar_setup(p.bar, slot, p.wait_ticks)) return;
  uint32_t nbar = 0;
  for (int32_t round = 0; round < p.max_rounds; ++round) {
    // ---- phase 1: this workgroup's tiles of every active graph.  Global tile gi belongs to
    // workgroup gi % gridDim.x; the graphs' activity flags and first tiles are staged in LDS,
    // kBlock graphs at a time, so a stopped graph costs one LDS read.
    for (int32_t g0 = 0; g0 < p.G; g0 += kBlock) {
      const int32_t ng = min(kBlock, p.G - g0);
      __syncthreads();
      if (t < ng) {
        s_act[t] = p.states[g0 + t].active;
        s_base[t] = p.tile_base[g0 + t];
      }
      if (t == 0) s_base[ng] = p.tile_base[g0 + ng];
      __syncthreads();
      for (int32_t k = 0; k < ng; ++k) {
        if (!s_act[k]) continue;
        const int32_t base = s_base[k], end = s_base[k + 1];
        const int32_t first = base + ((blk - base) % nblk + nblk) % nblk;
        if (first >= end) continue;
        const int32_t g = g0 + k;
        const MultiGraph &mg = p.graphs[g];
        const MultiGraphState &gs = p.states[g];
        const int par = gs.iters & 1;
        TileCtx<double> c{};
        c.off = mg.off;
        c.idx = mg.idx;
        c.outdeg = mg.outdeg;
        c.yin = mg.y[par];
        c.xs = c.yin;
        c.yout = mg.y[par ^ 1];
        c.hpart = mg.hpart;
        c.c0 = gs.c0;
        c.alpha = mg.alpha;
        c.mid_deg = mg.mid_deg;
        Acc a = {0.0, 0.0, 0.0, 0.0};
        for (int32_t gi = first; gi < end; gi += nblk) update_tile<double>(c, mg.desc[gi - base], mg.desc[gi - base + 1], a, vals, red);
        flush_acc(p, (int64_t)mg.pslot + (first - base), a, red);
      }
    }
    if (!grid_barrier(p.bar, slot, ++nbar, p.wait_ticks)) break;

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
        const double *bp = p.part + ((int64_t)mg.pslot + k) * 4;
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
    if (!grid_barrier(p.bar, slot, ++nbar, p.wait_ticks)) break;
    // every lane reads a strided share of the flags; the block ORs them
    int any = 0;
    for (int g = t; g < p.G; g += kBlock) any |= p.states[g].active;
    if (!__syncthreads_or(any)) break;
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
  if (threadIdx.x == 0) p.init_part[(int64_t)g * gridDim.x + blockIdx.x] = dang;
}

__global__ __launch_bounds__(kBlock) void k_multi_init_finish(MultiParams p, int32_t nb) {
  __shared__ double red[kWaves];
  const int g = blockIdx.x;
  const MultiGraph &mg = p.graphs[g];
  double D = 0.0;
  for (int32_t b = threadIdx.x; b < nb; b += kBlock) D += p.init_part[(int64_t)g * nb + b];
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
