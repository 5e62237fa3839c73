// batch.hip -- K rank columns of one graph in one pass over its edges (paper, section 2
// update, run for several damping factors / tolerances / error functions at once).
//
// State: Y[N][KP] in the phase's type VT (row width KP = 1, 2, 4, 8, 12 or 16 values, at most
// 16 columns), row-major, so one in-edge u -> v costs one contiguous KP*sizeof(VT)-byte row fetch
// that serves every column: y[u][k] = r_k[u]/d_u (or r_k[u] for a dangling u), as in pull.hip.
// A group of G = min(KP, 4) lanes owns one row fetch; lane (l % G) handles columns
// (l % G)*C .. +C-1, C = KP/G.
//   tiles of short rows (partition B: fewer than kSpanB entries): every group fetches the rows
//   of kPerQ entries into LDS, then one group sums each row of in-degree <= mid_deg in ascending
//   entry order and one wave each longer row (entry j on group j % (64/G), xor reduction);
//   long-row segments: one block per segment, reduction across groups and waves; hubs leave
//   per-column segment partials for k_batch_finish.
// Every column has its own c0, alpha, tau, norm, iteration count and stop decision; a column
// that stops is masked (no writes) and keeps its last iterate in the buffer given by its own
// update parity.  k_batch_hubs finishes the rows of several segments (16 rows per workgroup);
// k_batch_finish (one block) reduces the update and hub partials per column in block order and
// finalizes every active column.
#include "batch.h"

namespace prpull {

// Sum (max) over the 64/G groups of G lanes in a wave; lanes with equal (lane % G) end with
// equal bits.
template <int G, typename T>
__device__ __forceinline__ T xor_sum_groups(T v) {
#pragma unroll
  for (int o = G; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int G>
__device__ __forceinline__ double xor_max_groups(double v) {
#pragma unroll
  for (int o = G; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Lanes per row fetch and columns per lane of a row width.
template <int KP>
struct RowShape {
  static_assert(KP == 1 || KP == 2 || KP == 4 || KP == 8 || KP == 12 || KP == 16, "row width");
  static constexpr int G = KP < 4 ? KP : 4;
  static constexpr int C = KP / G;
};

template <typename VT, int C>
struct Row {
  VT v[C];
};

template <typename VT, int C>
__device__ __forceinline__ Row<VT, C> load_row(const VT *__restrict__ y, int32_t u, int kp, int c0) {
  Row<VT, C> r;
  const VT *p = y + (int64_t)u * kp + c0;
#pragma unroll
  for (int c = 0; c < C; ++c) r.v[c] = p[c];
  return r;
}

struct BAcc {
  double l1, sq, mx, dang;
};

// Per-column epilogue of one row for the lane's C columns; yo holds the row's current values of
// those columns (fetched by the caller, in the tile path together with the gathered rows).
// c0 and alpha point at the teleport terms and damping factors of the lane's C columns.
template <typename VT, int C, typename VI = VT>
__device__ __forceinline__ void batch_epilogue(int32_t v, const double (&s)[C], int32_t dv, const VI (&yold)[C],
                                               VT *__restrict__ yout, int kp, int col0, const double *c0,
                                               const double *alpha, const bool (&act)[C], BAcc (&a)[C]) {
#pragma clang fp contract(off)
  const int64_t base = (int64_t)v * kp + col0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    if (!act[c]) continue;
    const double rn = c0[c] + alpha[c] * s[c];
    const VT yo = (VT)yold[c];
    double old, rnew;
    if (dv > 0) {
      old = (double)yo * (double)dv;
      const VT y = (VT)(rn / (double)dv);
      yout[base + c] = y;
      rnew = sizeof(VT) == 8 ? rn : (double)y * (double)dv;
    } else {
      old = (double)yo;
      const VT y = (VT)rn;
      yout[base + c] = y;
      rnew = (double)y;
      a[c].dang += rnew;
    }
    const double d = fabs(rnew - old);
    a[c].l1 += d;
    a[c].sq += d * d;
    a[c].mx = fmax(a[c].mx, d);
  }
}

// Waves per SIMD the float32 update of a row width is compiled for (its registers are capped to
// fit them; one workgroup puts one wave on each SIMD).  The update is bound by row fetches in
// flight, so more resident waves pay as long as the cap forces only a small spill (12-20 bytes
// per lane at these settings); 12 values at 6 waves and 8 values at 8 spilled more and lost, and
// LDS admits no more than 4 workgroups of 16 values.  Measured on the scale-24 R-MAT alpha
// sweep; 1 = no cap (1 and 2 values stay under 64 registers by themselves; float64 rows are
// bound by LDS first).
// The first float64 update of a mixed batch reads the float32 rows of the handover (VI = float,
// exact in float64) and sums in float64.
constexpr int kF32RowsWaves = 1;

template <typename VT, int KP, typename VI = VT>
constexpr int update_waves() {
  return sizeof(VT) != 4 ? (sizeof(VI) == 4 ? kF32RowsWaves : 1) : KP == 16 ? 4 : KP == 12 ? 5 : KP == 8 ? 6 : KP == 4 ? 7 : 1;
}

template <typename VT, int KP, typename VI = VT>
__global__ __launch_bounds__(kBlock, (update_waves<VT, KP, VI>())) void k_batch_update(BatchParams p) {
  constexpr int G = RowShape<KP>::G, C = RowShape<KP>::C;
  constexpr int kQuads = kBlock / G;                        // groups per block (64, 128, 256)
  constexpr int kGW = 64 / G;                               // groups per wave
  constexpr int kPerQ = kSpanB / kQuads;                    // entries gathered per group per tile (8, 4, 2)
  constexpr int kRowsQ = (kRowsB + kQuads - 1) / kQuads;    // rows owned per group per tile (2, 1, 1)
  __shared__ VI vals[kSpanB * KP];
  __shared__ double sred[kWaves][KP];
  __shared__ double sacc[kWaves][KP][4];
  __shared__ double sc0[KP], salpha[KP];  // per-column terms in LDS rather than 2*C registers
  const BatchState *st = p.st;
  if (st->head.stop) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int qp = lane % G, quad = t / G;  // lane within its group, group in the block
  const int col0 = qp * C;
  if (t < KP) {
    sc0[t] = st->col[t].c0;
    salpha[t] = p.cols->alpha[t];
  }
  bool act[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int k = col0 + c;
    act[c] = k < p.K && st->col[k].active;
  }
  const double *c0 = sc0 + col0, *alpha = salpha + col0;
  __syncthreads();
  const VI *__restrict__ yin = (const VI *)p.y_in;
  VT *__restrict__ yout = (VT *)p.y_out;
  const int32_t *__restrict__ off = p.off;
  const int32_t *__restrict__ idx = p.idx;
  BAcc a[C];
#pragma unroll
  for (int c = 0; c < C; ++c) a[c] = BAcc{0.0, 0.0, 0.0, 0.0};

  for (int32_t i = blockIdx.x; i < p.ndesc; i += gridDim.x) {
    const int4 d = p.desc[i];
    const int4 dn = p.desc[i + 1];
    const int32_t e0 = d.y, e1 = dn.y;
    if (d.z < 0) {
      // ---- tile of short rows [d.x, dn.x), entries [e0, e1), fewer than kSpanB.
      // Phase 1: every quad fetches the rows of kPerQ entries (entry j on quad j % 64) and the
      // metadata of its rows; phase 2: row sums from LDS, one quad per short row, one wave per
      // mid row; then the epilogue.
      const int32_t v0 = d.x, v1 = dn.x, n = e1 - e0;
      int32_t u[kPerQ];
#pragma unroll
      for (int k = 0; k < kPerQ; ++k) {
        const int32_t j = quad + k * kQuads;
        u[k] = j < n ? __builtin_nontemporal_load(idx + e0 + j) : -1;
      }
      int32_t ra[kRowsQ], rb[kRowsQ], dv[kRowsQ];
#pragma unroll
      for (int q = 0; q < kRowsQ; ++q) {
        const int32_t v = v0 + quad + q * kQuads;
        ra[q] = rb[q] = dv[q] = 0;
        if (v < v1) {
          ra[q] = __builtin_nontemporal_load(off + v) - e0;
          rb[q] = __builtin_nontemporal_load(off + v + 1) - e0;
          dv[q] = __builtin_nontemporal_load(p.outdeg + v);
        }
      }
      Row<VI, C> x[kPerQ];
#pragma unroll
      for (int k = 0; k < kPerQ; ++k) {
        if (u[k] >= 0) {
          x[k] = load_row<VI, C>(yin, u[k], KP, col0);
        } else {
#pragma unroll
          for (int c = 0; c < C; ++c) x[k].v[c] = (VI)0;
        }
      }
      // the current values of the group's own rows, in flight with the gather (the epilogue
      // would otherwise wait for them after the row sums)
      Row<VI, C> yo[kRowsQ];
#pragma unroll
      for (int q = 0; q < kRowsQ; ++q) {
        const int32_t v = v0 + quad + q * kQuads;
        if (v < v1) {
          yo[q] = load_row<VI, C>(yin, v, KP, col0);
        } else {
#pragma unroll
          for (int c = 0; c < C; ++c) yo[q].v[c] = (VI)0;
        }
      }
#pragma unroll
      for (int k = 0; k < kPerQ; ++k) {
        const int32_t j = quad + k * kQuads;
        if (j < n) {
#pragma unroll
          for (int c = 0; c < C; ++c) vals[j * KP + col0 + c] = x[k].v[c];
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kRowsQ; ++q) {
        const int32_t v = v0 + quad + q * kQuads;
        const bool mine = v < v1;
        const bool mid = mine && (rb[q] - ra[q]) > p.mid_deg;
        if (mine && !mid) {
          VT s[C];
#pragma unroll
          for (int c = 0; c < C; ++c) s[c] = (VT)0;
          for (int32_t j = ra[q]; j < rb[q]; ++j) {
#pragma unroll
            for (int c = 0; c < C; ++c) s[c] += vals[j * KP + col0 + c];
          }
          double sd[C];
#pragma unroll
          for (int c = 0; c < C; ++c) sd[c] = (double)s[c];
          batch_epilogue<VT, C, VI>(v, sd, dv[q], yo[q].v, yout, KP, col0, c0, alpha, act, a);
        }
        unsigned long long m = __ballot(mid && qp == 0);
        while (m) {
          const int src = __ffsll((long long)m) - 1;
          m &= m - 1;
          const int32_t wa = __shfl(ra[q], src, 64), wb = __shfl(rb[q], src, 64);
          const int32_t wv = __shfl(v, src, 64), wd = __shfl(dv[q], src, 64);
          VT s[C];
#pragma unroll
          for (int c = 0; c < C; ++c) s[c] = (VT)0;
          for (int32_t j = wa + lane / G; j < wb; j += kGW) {
#pragma unroll
            for (int c = 0; c < C; ++c) s[c] += vals[j * KP + col0 + c];
          }
          double sd[C];
          VI wo[C];  // the row's current values, from the group that owns it
#pragma unroll
          for (int c = 0; c < C; ++c) {
            sd[c] = (double)xor_sum_groups<G>(s[c]);
            wo[c] = __shfl(yo[q].v[c], src + qp, 64);
          }
          if (lane < G) batch_epilogue<VT, C, VI>(wv, sd, wd, wo, yout, KP, col0, c0, alpha, act, a);
        }
      }
      __syncthreads();
    } else {
      // ---- one segment [e0, e1) of a long row: groups stride the entries, kPerQ in flight
      const int32_t v = d.x, slot = d.w;
      VT s[C];
#pragma unroll
      for (int c = 0; c < C; ++c) s[c] = (VT)0;
      for (int32_t c8 = e0 + quad; c8 < e1; c8 += kPerQ * kQuads) {
        int32_t u[kPerQ];
#pragma unroll
        for (int k = 0; k < kPerQ; ++k) {
          const int32_t j = c8 + k * kQuads;
          u[k] = j < e1 ? __builtin_nontemporal_load(idx + j) : -1;
        }
        Row<VI, C> x[kPerQ];
#pragma unroll
        for (int k = 0; k < kPerQ; ++k) {
          if (u[k] >= 0) {
            x[k] = load_row<VI, C>(yin, u[k], KP, col0);
          } else {
#pragma unroll
            for (int c = 0; c < C; ++c) x[k].v[c] = (VI)0;
          }
        }
#pragma unroll
        for (int k = 0; k < kPerQ; ++k) {
#pragma unroll
          for (int c = 0; c < C; ++c) s[c] += x[k].v[c];
        }
      }
      double tot[C];
#pragma unroll
      for (int c = 0; c < C; ++c) tot[c] = xor_sum_groups<G>((double)s[c]);
      __syncthreads();
      if (lane < G) {
#pragma unroll
        for (int c = 0; c < C; ++c) sred[wave][col0 + c] = tot[c];
      }
      __syncthreads();
      if (t < G) {
        double segd[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          double x = sred[0][col0 + c];
#pragma unroll
          for (int w = 1; w < kWaves; ++w) x += sred[w][col0 + c];
          segd[c] = x;
        }
        if (slot < 0) {
          // one-segment long row: finish here
          const Row<VI, C> o = load_row<VI, C>(yin, v, KP, col0);
          batch_epilogue<VT, C, VI>(v, segd, p.outdeg[v], o.v, yout, KP, col0, c0, alpha, act, a);
        } else {
#pragma unroll
          for (int c = 0; c < C; ++c) p.hpart[(int64_t)slot * KP + col0 + c] = segd[c];
        }
      }
    }
  }
  __syncthreads();

  // ---- block partials per column: lanes with equal qp reduce across groups and waves
#pragma unroll
  for (int c = 0; c < C; ++c) {
    a[c].l1 = xor_sum_groups<G>(a[c].l1);
    a[c].sq = xor_sum_groups<G>(a[c].sq);
    a[c].mx = xor_max_groups<G>(a[c].mx);
    a[c].dang = xor_sum_groups<G>(a[c].dang);
  }
  if (lane < G) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      sacc[wave][col0 + c][0] = a[c].l1;
      sacc[wave][col0 + c][1] = a[c].sq;
      sacc[wave][col0 + c][2] = a[c].mx;
      sacc[wave][col0 + c][3] = a[c].dang;
    }
  }
  __syncthreads();
  if (t < KP * 4) {
    const int k = t >> 2, f = t & 3;
    double x = sacc[0][k][f];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) x = f == 2 ? fmax(x, sacc[w][k][f]) : x + sacc[w][k][f];
    p.bpart[((int64_t)blockIdx.x * KP + k) * 4 + f] = x;
  }
}

// Hub rows: lane t of workgroup b finishes column t % 16 of hub row 16*b + t/16 (its segment
// sums in segment order, then the epilogue); the workgroup's per-column partials are combined over
// its 16 rows in row order and stored to hacc[b].
template <typename VT, int KP, typename VI = VT>
__global__ __launch_bounds__(kBlock) void k_batch_hubs(BatchParams p) {
  __shared__ double sacc[kHubsPerBlock][16][4];
  const BatchState *st = p.st;
  if (st->head.stop) return;
  const int t = threadIdx.x, k = t & 15, j = t >> 4;
  const int32_t h = (int32_t)blockIdx.x * kHubsPerBlock + j;
  BAcc a = {0.0, 0.0, 0.0, 0.0};
  if (h < p.nhubs && k < p.K && k < KP && st->col[k].active) {
    const VI *__restrict__ yin = (const VI *)p.y_in;
    VT *__restrict__ yout = (VT *)p.y_out;
    const double c0 = st->col[k].c0, alpha = p.cols->alpha[k];
    const int4 hb = p.hubs[h];
    double s = 0.0;
#pragma unroll 1
    for (int32_t q = 0; q < hb.y; ++q) s += p.hpart[(int64_t)(hb.z + q) * KP + k];
    double sv[1] = {s};
    bool act[1] = {true};
    BAcc aa[1] = {a};
    // the epilogue addresses column k of row hb.x
    const VI yo[1] = {yin[(int64_t)hb.x * KP + k]};
    batch_epilogue<VT, 1, VI>(hb.x, sv, p.outdeg[hb.x], yo, yout, KP, k, &c0, &alpha, act, aa);
    a = aa[0];
  }
  sacc[j][k][0] = a.l1;
  sacc[j][k][1] = a.sq;
  sacc[j][k][2] = a.mx;
  sacc[j][k][3] = a.dang;
  __syncthreads();
  if (t < KP * 4) {
    const int col = t >> 2, f = t & 3;
    double x = sacc[0][col][f];
#pragma unroll 1
    for (int r = 1; r < kHubsPerBlock; ++r) x = f == 2 ? fmax(x, sacc[r][col][f]) : x + sacc[r][col][f];
    p.hacc[((int64_t)blockIdx.x * KP + col) * 4 + f] = x;
  }
}

// One block of kFinBlock lanes: lane t works on column t % 16 (columns >= Kp idle) and adds the
// partials of the update workgroups, then those of the hub workgroups, each in block order.
template <typename VT, int KP>
__global__ __launch_bounds__(kFinBlock) void k_batch_finish(BatchParams p) {
  constexpr int kGroups = kFinBlock / 16;
  __shared__ double sacc[kGroups][16][4];
  BatchState *st = p.st;
  if (st->head.stop) return;
  const int t = threadIdx.x, k = t & 15, g = t >> 4;
  BAcc a = {0.0, 0.0, 0.0, 0.0};
  const bool col = k < p.K && k < KP && st->col[k].active;
  if (col) {
    for (int32_t b = g; b < p.grid; b += kGroups) {
      const double *bp = p.bpart + ((int64_t)b * KP + k) * 4;
      a.l1 += bp[0];
      a.sq += bp[1];
      a.mx = fmax(a.mx, bp[2]);
      a.dang += bp[3];
    }
    const int32_t nhb = (int32_t)hub_blocks(p.nhubs);
    for (int32_t b = g; b < nhb; b += kGroups) {
      const double *bp = p.hacc + ((int64_t)b * KP + k) * 4;
      a.l1 += bp[0];
      a.sq += bp[1];
      a.mx = fmax(a.mx, bp[2]);
      a.dang += bp[3];
    }
  }
  sacc[g][k][0] = a.l1;
  sacc[g][k][1] = a.sq;
  sacc[g][k][2] = a.mx;
  sacc[g][k][3] = a.dang;
  __syncthreads();
  if (t < 16) {
    double l1 = 0.0, sq = 0.0, mx = 0.0, dang = 0.0;
#pragma unroll 1
    for (int gg = 0; gg < kGroups; ++gg) {
      l1 += sacc[gg][t][0];
      sq += sacc[gg][t][1];
      mx = fmax(mx, sacc[gg][t][2]);
      dang += sacc[gg][t][3];
    }
    if (t < p.K && st->col[t].active) batch_finalize_column(p, t, l1, sq, mx, dang);
  }
  __syncthreads();
  if (t == 0) {
    int any = 0, all_done = 1;
#pragma unroll 1
    for (int c = 0; c < p.K; ++c) {
      any |= st->col[c].active;
      all_done &= st->col[c].done;
    }
    st->head.iter += 1;
    st->head.phase_iter += 1;
    st->head.stop = !any;
    st->head.done = all_done;
  }
}

// Grid-stride lanes over a row-major [N][kp] array in which every lane keeps one column: the
// stride is the largest multiple of kp within the grid's lane count, so consecutive lanes touch
// consecutive elements and no lane divides inside its loop.
struct ColLane {
  int64_t v;      // first row
  int64_t vstep;  // rows per grid sweep
  int c;          // the lane's column
  bool on;        // lanes past the last whole row of a sweep idle
};

__device__ __forceinline__ ColLane col_lane(int kp) {
  const int32_t lanes = (int32_t)(gridDim.x * blockDim.x);
  const int32_t per = lanes / kp;
  const int32_t tid = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  ColLane r;
  r.on = tid < per * kp;
  r.v = tid / kp;
  r.c = tid % kp;
  r.vstep = per;
  return r;
}

// Start vectors: column k from init[k] (or 1/N); per-block, per-column dangling sums.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_batch_init(const int32_t *__restrict__ outdeg, int32_t N, int32_t K,
                                                       int32_t kp, BatchParams p, VT *__restrict__ y,
                                                       double *bpart) {
#pragma clang fp contract(off)
  __shared__ double s[kBlock];
  const ColLane cl = col_lane(kp);
  double dang = 0.0;
  if (cl.on) {
    const int c = cl.c;
    const double *ini = c < K ? p.cols->init[c] : nullptr;
    const double r1 = 1.0 / (double)N;
    for (int64_t v = cl.v; v < N; v += cl.vstep) {
      VT yy = (VT)0;
      if (c < K) {
        const int32_t dv = outdeg[v];
        const double r0 = ini ? ini[v] : r1;
        if (dv > 0) {
          yy = (VT)(r0 / (double)dv);
        } else {
          yy = (VT)r0;
          dang += (double)yy;
        }
      }
      y[v * kp + c] = yy;
    }
  }
  s[threadIdx.x] = dang;
  __syncthreads();
  // per column: the block's lanes of that column in lane order
  if (threadIdx.x < 16) {
    const int t = threadIdx.x;
    double x = 0.0;
    if (t < kp) {
      const int base = (int)(((int64_t)blockIdx.x * kBlock) % kp);
      for (int i = (t - base + kp) % kp; i < kBlock; i += kp) x += s[i];
    }
    bpart[(int64_t)blockIdx.x * 16 + t] = x;
  }
}

__global__ __launch_bounds__(kFinBlock) void k_batch_init_finish(const double *__restrict__ bpart, int32_t nb,
                                                                 int32_t N, BatchParams p, int32_t phase) {
#pragma clang fp contract(off)
  constexpr int kGroups = kFinBlock / 16;
  __shared__ double s[kGroups][16];
  const int t = threadIdx.x, k = t & 15, g = t >> 4;
  double D = 0.0;
  for (int32_t b = g; b < nb; b += kGroups) D += bpart[(int64_t)b * 16 + k];
  s[g][k] = D;
  __syncthreads();
  BatchState *st = p.st;
  if (t < 16) {
    double x = 0.0;
#pragma unroll 1
    for (int i = 0; i < kGroups; ++i) x += s[i][t];
    BatchColumn &cs = st->col[t];
    const double Nd = (double)N;
    const double al = t < p.K ? p.cols->alpha[t] : 0.0;
    cs.c0 = (1.0 - al) / Nd + (al * x) / Nd;
    cs.iters = 0;
    cs.fp32_iters = 0;
    cs.phase_updates = 0;
    cs.converged = 0;
    cs.done = t < p.K ? 0 : 1;
    cs.active = t < p.K ? 1 : 0;
    cs.prev_l1 = __builtin_huge_val();
    cs.err[0] = cs.err[1] = cs.err[2] = 0.0;
  }
  if (t == 0) {
    st->head.iter = 0;
    st->head.phase_iter = 0;
    st->head.stop = 0;
    st->head.done = 0;
    st->phase = phase;
  }
}

// Float32 columns leaving the float32 phase -> column-major staging: column c (its newest buffer
// by its update parity) goes to ycol[map[c]][0..N) (skipped when map[c] < 0).  One lane per row,
// the columns in turn, so that each column's stores are contiguous: whole lines, where stores of
// single values into the float64 rows would rewrite every line of those rows in part.  The values
// stay float32 (their float64 value is exact).
__global__ __launch_bounds__(kBlock) void k_batch_convert(const float *__restrict__ y32a, const float *__restrict__ y32b,
                                                          int32_t kp32, float *__restrict__ ycol, int32_t N, int32_t K,
                                                          const BatchState *st, const BatchCols *cols) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock) {
    for (int c = 0; c < K; ++c) {
      const int d = cols->map[c];
      if (d < 0) continue;
      const float *__restrict__ src = (st->col[c].phase_updates & 1) ? y32b : y32a;
      ycol[(int64_t)d * N + v] = src[v * kp32 + c];
    }
  }
}

// Staging ycol[K][N] -> rows y[N][kp] of the float64 phase (padding columns zero), as float64 or
// as the float32 values themselves, through an LDS tile of kRowsT rows so that reads and stores
// are both contiguous.
constexpr int kRowsT = 64;
template <typename VO>
__global__ __launch_bounds__(kBlock) void k_batch_rows(const float *__restrict__ ycol, VO *__restrict__ y64,
                                                       int32_t kp64, int32_t N, int32_t K) {
  __shared__ float tile[16][kRowsT + 1];
  for (int64_t v0 = (int64_t)blockIdx.x * kRowsT; v0 < N; v0 += (int64_t)gridDim.x * kRowsT) {
    const int rows = (int)(N - v0 < kRowsT ? N - v0 : kRowsT);
    for (int i = threadIdx.x; i < kp64 * kRowsT; i += kBlock) {
      const int k = i / kRowsT, r = i % kRowsT;
      if (r < rows) tile[k][r] = k < K ? ycol[(int64_t)k * N + v0 + r] : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < rows * kp64; i += kBlock) {
      const int r = i / kp64, k = i % kp64;
      y64[(v0 + r) * kp64 + k] = (VO)tile[k][r];
    }
    __syncthreads();
  }
}

// Repack: column i of dst (i < K) is column map[i] of src; padding columns are zero.  Lanes keep
// one destination column, in memory order.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_batch_compact(const VT *__restrict__ src, int32_t kp_src,
                                                          VT *__restrict__ dst, int32_t kp_dst, int32_t N, int32_t K,
                                                          const BatchCols *cols) {
  const ColLane cl = col_lane(kp_dst);
  if (!cl.on) return;
  const int c = cl.c, m = c < K ? cols->map[c] : -1;
  for (int64_t v = cl.v; v < N; v += cl.vstep) dst[v * kp_dst + c] = m >= 0 ? src[v * kp_src + m] : (VT)0;
}

// Re-arm for the float64 phase: every column not done becomes active.
__global__ void k_batch_rearm(BatchState *st, int32_t K) {
  if (threadIdx.x == 0) {
    int any = 0;
    for (int c = 0; c < K; ++c) {
      BatchColumn &cs = st->col[c];
      cs.phase_updates = 0;
      cs.active = !cs.done;
      any |= cs.active;
    }
    st->head.phase_iter = 0;
    st->head.stop = !any;
    st->phase = 2;
  }
}

// ranks[k][v] from the buffer holding column k's newest iterate.  A block moves tiles of
// kOutRows rows through LDS: read in memory order (lanes keep one column), written one column
// per wave, 64 consecutive vertices at a time.
constexpr int kOutRows = 64;
constexpr int kOutPitch = kMaxCols + 1;  // odd pitch in doubles: the column reads are conflict-free
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_batch_output(const int32_t *__restrict__ outdeg, const VT *__restrict__ ya,
                                                         const VT *__restrict__ yb, int32_t kp, int32_t N, int32_t K,
                                                         BatchParams p) {
  __shared__ double tile[kOutRows * kOutPitch];
  const BatchState *st = p.st;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int rc = t % kp, rr = t / kp, rstep = kBlock / kp;  // load phase: lane (row rr, column rc)
  const bool ld = rr < rstep && rc < K;
  const VT *__restrict__ src = ld && (st->col[rc].phase_updates & 1) ? yb : ya;
  for (int64_t v0 = (int64_t)blockIdx.x * kOutRows; v0 < N; v0 += (int64_t)gridDim.x * kOutRows) {
    const int rows = (int)(N - v0 < kOutRows ? N - v0 : kOutRows);
    if (ld) {
      for (int r = rr; r < rows; r += rstep) tile[r * kOutPitch + rc] = (double)src[(v0 + r) * kp + rc];
    }
    __syncthreads();
    if (lane < rows) {
      const int32_t dv = outdeg[v0 + lane];
      for (int c = wave; c < K; c += kWaves) {
        double *out = p.cols->ranks[c];
        if (!out) continue;
        const double y = tile[lane * kOutPitch + c];
        out[v0 + lane] = dv > 0 ? y * (double)dv : y;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ launchers
static unsigned grid_for(int64_t n, int64_t cap) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

static unsigned out_grid(int64_t N) {
  const int64_t tiles = (N + kOutRows - 1) / kOutRows;
  return (unsigned)(tiles < 1 ? 1 : tiles > 4096 ? 4096 : tiles);
}

template <typename VT, int KP, typename VI = VT>
static void batch_update_w(hipStream_t s, unsigned grid, const BatchParams &p) {
  hipLaunchKernelGGL((k_batch_update<VT, KP, VI>), dim3(grid), dim3(kBlock), 0, s, p);
  if (p.nhubs > 0) hipLaunchKernelGGL((k_batch_hubs<VT, KP, VI>), dim3(hub_blocks(p.nhubs)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL((k_batch_finish<VT, KP>), dim3(1), dim3(kFinBlock), 0, s, p);
}

template <typename VT>
static hipError_t batch_update_t(hipStream_t s, int kp, unsigned grid, const BatchParams &p) {
  switch (kp) {
    case 1: batch_update_w<VT, 1>(s, grid, p); break;
    case 2: batch_update_w<VT, 2>(s, grid, p); break;
    case 4: batch_update_w<VT, 4>(s, grid, p); break;
    case 8: batch_update_w<VT, 8>(s, grid, p); break;
    case 12: batch_update_w<VT, 12>(s, grid, p); break;
    case 16: batch_update_w<VT, 16>(s, grid, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_update(hipStream_t s, bool fp32, int kp, unsigned grid, const BatchParams &p) {
  return fp32 ? batch_update_t<float>(s, kp, grid, p) : batch_update_t<double>(s, kp, grid, p);
}

hipError_t launch_batch_update_f32rows(hipStream_t s, int kp, unsigned grid, const BatchParams &p) {
  switch (kp) {
    case 1: batch_update_w<double, 1, float>(s, grid, p); break;
    case 2: batch_update_w<double, 2, float>(s, grid, p); break;
    case 4: batch_update_w<double, 4, float>(s, grid, p); break;
    case 8: batch_update_w<double, 8, float>(s, grid, p); break;
    case 12: batch_update_w<double, 12, float>(s, grid, p); break;
    case 16: batch_update_w<double, 16, float>(s, grid, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename VT>
static int blocks_per_cu_t(int kp) {
  int n = 0;
  hipError_t e;
  switch (kp) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<VT, 1>, kBlock, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<VT, 2>, kBlock, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<VT, 4>, kBlock, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<VT, 8>, kBlock, 0); break;
    case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<VT, 12>, kBlock, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<VT, 16>, kBlock, 0); break;
  }
  return e == hipSuccess && n > 0 ? n : 1;
}

int batch_blocks_per_cu(bool fp32, int kp) { return fp32 ? blocks_per_cu_t<float>(kp) : blocks_per_cu_t<double>(kp); }

int batch_blocks_per_cu_f32rows(int kp) {
  int n = 0;
  hipError_t e;
  switch (kp) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<double, 1, float>, kBlock, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<double, 2, float>, kBlock, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<double, 4, float>, kBlock, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<double, 8, float>, kBlock, 0); break;
    case 12: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<double, 12, float>, kBlock, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_update<double, 16, float>, kBlock, 0); break;
  }
  return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_batch_init(hipStream_t s, bool fp32, const int32_t *outdeg, int32_t N, int32_t K, int32_t kp,
                             void *y, double *bpart, int64_t bpart_blocks, const BatchParams &p, int32_t phase) {
  const unsigned g = grid_for((int64_t)N * kp, bpart_blocks < 2048 ? bpart_blocks : 2048);
  if (fp32)
    hipLaunchKernelGGL(k_batch_init<float>, dim3(g), dim3(kBlock), 0, s, outdeg, N, K, kp, p, (float *)y, bpart);
  else
    hipLaunchKernelGGL(k_batch_init<double>, dim3(g), dim3(kBlock), 0, s, outdeg, N, K, kp, p, (double *)y, bpart);
  hipLaunchKernelGGL(k_batch_init_finish, dim3(1), dim3(kFinBlock), 0, s, (const double *)bpart, (int32_t)g, N, p,
                     phase);
  return hipGetLastError();
}

hipError_t launch_batch_convert(hipStream_t s, const float *y32a, const float *y32b, int32_t kp32, float *ycol,
                                int32_t N, int32_t K, const BatchState *st, const BatchCols *cols) {
  hipLaunchKernelGGL(k_batch_convert, dim3(grid_for(N, 8192)), dim3(kBlock), 0, s, y32a, y32b, kp32, ycol, N, K, st,
                     cols);
  return hipGetLastError();
}

hipError_t launch_batch_rows(hipStream_t s, const float *ycol, void *y, bool f64, int32_t kp, int32_t N, int32_t K) {
  if (kp < 1 || kp > 16 || K > kp) return hipErrorInvalidValue;
  const int64_t tiles = ((int64_t)N + kRowsT - 1) / kRowsT;
  const dim3 grid((unsigned)(tiles < 1 ? 1 : tiles > 8192 ? 8192 : tiles));
  if (f64)
    hipLaunchKernelGGL(k_batch_rows<double>, grid, dim3(kBlock), 0, s, ycol, (double *)y, kp, N, K);
  else
    hipLaunchKernelGGL(k_batch_rows<float>, grid, dim3(kBlock), 0, s, ycol, (float *)y, kp, N, K);
  return hipGetLastError();
}

hipError_t launch_batch_rearm(hipStream_t s, BatchState *st, int32_t K) {
  hipLaunchKernelGGL(k_batch_rearm, dim3(1), dim3(64), 0, s, st, K);
  return hipGetLastError();
}

hipError_t launch_batch_compact(hipStream_t s, bool fp32, const void *src, int32_t kp_src, void *dst, int32_t kp_dst,
                                int32_t N, int32_t K, const BatchCols *cols) {
  if (fp32)
    hipLaunchKernelGGL(k_batch_compact<float>, dim3(grid_for((int64_t)N * kp_dst, 8192)), dim3(kBlock), 0, s,
                       (const float *)src, kp_src, (float *)dst, kp_dst, N, K, cols);
  else
    hipLaunchKernelGGL(k_batch_compact<double>, dim3(grid_for((int64_t)N * kp_dst, 8192)), dim3(kBlock), 0, s,
                       (const double *)src, kp_src, (double *)dst, kp_dst, N, K, cols);
  return hipGetLastError();
}

hipError_t launch_batch_output(hipStream_t s, bool fp32, const int32_t *outdeg, const void *ya, const void *yb,
                               int32_t kp, int32_t N, int32_t K, const BatchParams &p) {
  if (fp32)
    hipLaunchKernelGGL(k_batch_output<float>, dim3(out_grid(N)), dim3(kBlock), 0, s, outdeg,
                       (const float *)ya, (const float *)yb, kp, N, K, p);
  else
    hipLaunchKernelGGL(k_batch_output<double>, dim3(out_grid(N)), dim3(kBlock), 0, s, outdeg,
                       (const double *)ya, (const double *)yb, kp, N, K, p);
  return hipGetLastError();
}

}  // namespace prpull
