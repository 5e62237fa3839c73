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
//   sum      : one lane per low in-degree row, one wave64 per mid row, fixed-order block
//              reduction per hub segment and a fixed-order combine by the last segment;
//   epilogue : r'_v = c0 + alpha*s_v, the new y_v, |r'_v - r_v| into L1/L2/Linf partials and
//              r'_v of dangling vertices into the dangling-sum partial;
//   finalize : the last block to finish reduces the block partials in block order and sets
//              the errors, the next teleport term c0 = (1-alpha)/N + (alpha*D)/N, the stop flags
//              and the trace row.
// Every reduction has a fixed order, so results are bitwise repeatable run to run.
#include "internal.h"

namespace prpull {

// ------------------------------------------------------------------ wave / block reductions
// xor butterflies: partners add the same two operands, so every lane ends with the same bits.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the block in a fixed order; the result is valid in every lane.
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = lds[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) s += lds[i];
  return s;
}

// ------------------------------------------------------------------ row epilogue
struct Acc {
  double l1, sq, mx, dang;
};

template <typename VT>
__device__ __forceinline__ void epilogue(int32_t v, double s, double c0, double alpha,
                                         const int32_t *__restrict__ outdeg, const VT *__restrict__ yin,
                                         VT *__restrict__ yout, Acc &a) {
#pragma clang fp contract(off)
  const double rn = c0 + alpha * s;
  const int32_t dv = outdeg[v];
  const VT yo = yin[v];
  double old, rnew;
  if (dv > 0) {
    old = (double)yo * (double)dv;
    const VT y = (VT)(rn / (double)dv);
    yout[v] = y;
    rnew = sizeof(VT) == 8 ? rn : (double)y * (double)dv;
  } else {
    old = (double)yo;
    const VT y = (VT)rn;
    yout[v] = y;
    rnew = (double)y;
    a.dang += rnew;
  }
  const double d = fabs(rnew - old);
  a.l1 += d;
  a.sq += d * d;
  a.mx = fmax(a.mx, d);
}

// Finalize one update: called by every lane of the last block, with the reduced totals.
__device__ __forceinline__ void finalize(const IterParams &p, double l1, double sq, double mx, double dang) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  SolveState *st = p.st;
  const double e[3] = {l1, sqrt(sq), mx};
  st->err[0] = e[0];
  st->err[1] = e[1];
  st->err[2] = e[2];
  const int32_t it = st->iter + 1;
  st->iter = it;
  st->phase_iter = st->phase_iter + 1;
  if (p.trace) {
    p.trace[3 * (int64_t)(it - 1) + 0] = e[0];
    p.trace[3 * (int64_t)(it - 1) + 1] = e[1];
    p.trace[3 * (int64_t)(it - 1) + 2] = e[2];
  }
  const double N = (double)p.N;
  st->c0 = (1.0 - p.alpha) / N + (p.alpha * dang) / N;
  const bool met = e[p.norm - 1] < p.tau;
  if (p.phase == 1) {
    // float32 phase: hand over to float64 once tau is met or the L1 change stops shrinking
    // (in exact arithmetic the L1 change never grows: the update is an alpha-contraction in L1)
    if (met) st->met32 = 1;
    if (met || !(l1 < st->prev_l1)) st->stop = 1;
    st->prev_l1 = l1;
    if (it >= p.max_iter) {
      st->stop = 1;
      st->done = 1;
    }
  } else {
    if (met) {
      st->converged = 1;
      st->stop = 1;
      st->done = 1;
    } else if (it >= p.max_iter) {
      st->stop = 1;
      st->done = 1;
    }
  }
  st->ticket = 0;
}

// ------------------------------------------------------------------ the update kernel
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_update(IterParams p) {
  __shared__ VT vals[kSpan];
  __shared__ double red[kWaves];
  __shared__ int s_last;
  const SolveState *st = p.st;
  if (st->stop) return;
  const double c0 = st->c0;
  const double alpha = p.alpha;
  const VT *__restrict__ yin = (const VT *)p.y_in;
  VT *__restrict__ yout = (VT *)p.y_out;
  const int32_t *__restrict__ off = p.off;
  const int32_t *__restrict__ idx = p.idx;
  const int t = threadIdx.x, lane = t & 63;
  Acc a = {0.0, 0.0, 0.0, 0.0};

  for (int32_t i = blockIdx.x; i < p.ndesc; i += gridDim.x) {
    const int4 d = p.desc[i];
    if (d.z < 0) {
      // ---- tile of rows [v0, v1): stage the contributions of its entries into LDS
      const int32_t v0 = d.x, v1 = p.desc[i + 1].x;
      const int32_t e0 = off[v0];
      const int32_t n = off[v1] - e0;  // < kSpan
      constexpr int kPer = kSpan / kBlock;
      int32_t u[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int j = t + k * kBlock;
        u[k] = j < n ? idx[e0 + j] : -1;
      }
      VT x[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) x[k] = u[k] >= 0 ? yin[u[k]] : (VT)0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int j = t + k * kBlock;
        if (j < n) vals[j] = x[k];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kRowsPerLane; ++q) {
        const int32_t v = v0 + t + q * kBlock;
        const bool mine = v < v1;
        int32_t ra = 0, rb = 0;
        if (mine) {
          ra = off[v] - e0;
          rb = off[v + 1] - e0;
        }
        const bool mid = mine && (rb - ra) > kMidDeg;
        if (mine && !mid) {
          VT s = (VT)0;
          for (int32_t j = ra; j < rb; ++j) s += vals[j];
          epilogue<VT>(v, (double)s, c0, alpha, p.outdeg, yin, yout, a);
        }
        unsigned long long m = __ballot(mid);
        while (m) {
          const int src = __ffsll((long long)m) - 1;
          m &= m - 1;
          const int32_t wa = __shfl(ra, src, 64), wb = __shfl(rb, src, 64);
          VT s = (VT)0;
          for (int32_t j = wa + lane; j < wb; j += 64) s += vals[j];
          s = wave_sum(s);
          if (lane == src) epilogue<VT>(v, (double)s, c0, alpha, p.outdeg, yin, yout, a);
        }
      }
      __syncthreads();
    } else {
      // ---- one kTile-entry segment of a hub row
      const int32_t v = d.x, ns = d.y, sg = d.z, slot = d.w;
      const int32_t e0 = off[v] + sg * kTile;
      const int32_t e1 = min(e0 + kTile, off[v + 1]);
      const int32_t n = e1 - e0;
      constexpr int kPer = kTile / kBlock;
      int32_t u[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int j = t + k * kBlock;
        u[k] = j < n ? idx[e0 + j] : -1;
      }
      VT s = (VT)0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) s += u[k] >= 0 ? yin[u[k]] : (VT)0;
      const double seg = block_sum((double)s, red);
      if (t == 0) {
        p.hpart[slot + sg] = seg;
        __threadfence();
        const uint32_t tk = atomicAdd(&p.hcnt[slot], 1u);
        s_last = tk == (uint32_t)(ns - 1);
      }
      __syncthreads();
      if (s_last) {
        __threadfence();
        double h = 0.0;
        for (int32_t q = t; q < ns; q += kBlock) h += p.hpart[slot + q];
        h = block_sum(h, red);
        if (t == 0) {
          p.hcnt[slot] = 0;
          epilogue<VT>(v, h, c0, alpha, p.outdeg, yin, yout, a);
        }
      }
      __syncthreads();
    }
  }

  // ---- block partials, then the last block reduces them in block order
  const double l1 = block_sum(a.l1, red);
  const double sq = block_sum(a.sq, red);
  double mx = wave_max(a.mx);
  __syncthreads();
  if (lane == 0) red[t >> 6] = mx;
  __syncthreads();
  mx = red[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) mx = fmax(mx, red[i]);
  const double dang = block_sum(a.dang, red);
  if (t == 0) {
    double *bp = p.bpart + 4 * (int64_t)blockIdx.x;
    bp[0] = l1;
    bp[1] = sq;
    bp[2] = mx;
    bp[3] = dang;
    __threadfence();
    const uint32_t tk = atomicAdd(&p.st->ticket, 1u);
    s_last = tk == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double r1 = 0.0, r2 = 0.0, r3 = 0.0, r4 = 0.0;
  for (int32_t b = t; b < (int32_t)gridDim.x; b += kBlock) {
    const double *bp = p.bpart + 4 * (int64_t)b;
    r1 += bp[0];
    r2 += bp[1];
    r3 = fmax(r3, bp[2]);
    r4 += bp[3];
  }
  r1 = block_sum(r1, red);
  r2 = block_sum(r2, red);
  r4 = block_sum(r4, red);
  r3 = wave_max(r3);
  __syncthreads();
  if (lane == 0) red[t >> 6] = r3;
  __syncthreads();
  double m3 = red[0];
#pragma unroll
  for (int i = 1; i < kWaves; ++i) m3 = fmax(m3, red[i]);
  finalize(p, r1, r2, m3, r4);
}

// ------------------------------------------------------------------ init, convert, output
// y0 from the start vector (or 1/N), and c0 of the first update from its dangling sum.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_init(const int32_t *__restrict__ outdeg, int32_t N,
                                                 const double *__restrict__ init, VT *__restrict__ y,
                                                 double alpha, SolveState *st, double *bpart) {
#pragma clang fp contract(off)
  __shared__ double red[kWaves];
  __shared__ int s_last;
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
  if (threadIdx.x == 0) {
    bpart[blockIdx.x] = dang;
    __threadfence();
    s_last = atomicAdd(&st->ticket2, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double D = 0.0;
  for (int32_t b = threadIdx.x; b < (int32_t)gridDim.x; b += kBlock) D += bpart[b];
  D = block_sum(D, red);
  if (threadIdx.x == 0) {
    const double Nd = (double)N;
    st->c0 = (1.0 - alpha) / Nd + (alpha * D) / Nd;
    st->iter = 0;
    st->phase_iter = 0;
    st->stop = 0;
    st->done = 0;
    st->converged = 0;
    st->met32 = 0;
    st->prev_l1 = __builtin_huge_val();
    st->ticket = 0;
    st->ticket2 = 0;
  }
}

// Float32 iterate -> float64 iterate (same implied ranks), and re-arm the update kernels.
__global__ __launch_bounds__(kBlock) void k_convert(const float *__restrict__ y32, double *__restrict__ y64,
                                                    int32_t N, SolveState *st) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock)
    y64[v] = (double)y32[v];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->stop = st->done;
    st->phase_iter = 0;
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

// ------------------------------------------------------------------ launchers
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
    hipLaunchKernelGGL(k_init<float>, dim3(g), dim3(kBlock), 0, s, outdeg, N, init, (float *)y, alpha, st, bpart);
  else
    hipLaunchKernelGGL(k_init<double>, dim3(g), dim3(kBlock), 0, s, outdeg, N, init, (double *)y, alpha, st,
                       bpart);
  return hipGetLastError();
}

hipError_t launch_update(hipStream_t s, bool fp32, unsigned grid, const IterParams &p) {
  if (fp32)
    hipLaunchKernelGGL(k_update<float>, dim3(grid), dim3(kBlock), 0, s, p);
  else
    hipLaunchKernelGGL(k_update<double>, dim3(grid), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_convert(hipStream_t s, const float *y32, double *y64, int32_t N, SolveState *st) {
  hipLaunchKernelGGL(k_convert, dim3(grid_for(N, 2048)), dim3(kBlock), 0, s, y32, y64, N, st);
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
