// device.h -- device helpers shared by the update kernels (pull.hip, multi.hip).
#pragma once

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
__device__ __forceinline__ void epilogue(int32_t v, double s, double c0, double alpha, int32_t dv, VT yo,
                                         VT *__restrict__ yout, Acc &a) {
#pragma clang fp contract(off)
  const double rn = c0 + alpha * s;
  double old, rnew;
  if (dv > 0) {
    old = (double)yo * (double)dv;
    const VT y = (VT)(rn / (double)dv);
    __builtin_nontemporal_store(y, &yout[v]);
    rnew = sizeof(VT) == 8 ? rn : (double)y * (double)dv;
  } else {
    old = (double)yo;
    const VT y = (VT)rn;
    __builtin_nontemporal_store(y, &yout[v]);
    rnew = (double)y;
    a.dang += rnew;
  }
  const double d = fabs(rnew - old);
  a.l1 += d;
  a.sq += d * d;
  a.mx = fmax(a.mx, d);
}

// Fixed-order reduction over a block of NT lanes; every lane gets the result.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v, double *lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = lds[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) s += lds[i];
  return s;
}

template <int NT>
__device__ __forceinline__ double block_max_n(double v, double *lds) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = lds[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) s = fmax(s, lds[i]);
  return s;
}

// ------------------------------------------------------------------ one tile
// Everything one workgroup does for one tile descriptor d (dn is the next descriptor) of one
// graph in one update; the row epilogues accumulate into a (per lane).
// Rows are summed over xs[idx[j]]: xs is the iterate itself in the plain update; in the merge
// step of the source-segmented update it is the array of per-segment partial sums, idx listing a
// row's partial sums in segment order.  yin (the row's own current value) and yout serve the
// epilogue.  With Part = true a row's sum is stored as it is into part[row] (the per-segment
// step of the source-segmented update: rows are then (segment, row) pairs, no epilogue; a tile's
// indices may come in source order, packed with the pair-order position each gathered value is
// staged at, so every pair is summed in its own order).
template <typename VT>
struct TileCtx {
  const int32_t *off;
  const int32_t *idx;
  const int32_t *outdeg;
  const VT *xs;
  const VT *yin;
  VT *yout;
  VT *part;
  double *hpart;
  double c0;
  double alpha;
  int32_t mid_deg;  // rows with more entries are summed by a whole wave
};

// A pair's partial sum (the per-segment step): float64 partials are stored nontemporally (0.7%
// faster per update on R-MAT scale 24: they need not displace the segment's slice of the iterate
// from L2), float32 ones plainly (0.8% slower the other way).
template <typename VT>
__device__ __forceinline__ void store_partial(VT *p, VT s) {
  if constexpr (sizeof(VT) == 8)
    __builtin_nontemporal_store(s, p);
  else
    *p = s;
}

template <typename VT, bool Part = false>
__device__ __forceinline__ void update_tile(const TileCtx<VT> &c, const int4 d, const int4 dn, Acc &a, VT *vals,
                                            double *red) {
  const int t = threadIdx.x, lane = t & 63;
  constexpr int kPer = kSpan / kBlock;
  const int32_t *__restrict__ off = c.off;
  const int32_t *__restrict__ idx = c.idx;
  const VT *__restrict__ xs = c.xs;
  const VT *__restrict__ yin = c.yin;
  VT *__restrict__ yout = c.yout;
  const int32_t e0 = d.y, e1 = dn.y;
  if (d.z < 0) {
    // ---- tile of short rows [d.x, dn.x) with entries [e0, e1), e1 - e0 < kSpan.
    // One round trip for the index stream and the rows' own data, one for the gather.
    const int32_t v0 = d.x, v1 = dn.x;
    const int32_t n = e1 - e0;
    // Part: a tile with d.w >= 0 lists its entries in source order, each word packing the
    // source less d.w and the entry's pair-order position (where its value is staged)
    const int32_t base = Part ? d.w : -1;
    int32_t u[kPer], pk[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = t + k * kBlock;
      u[k] = j < n ? __builtin_nontemporal_load(idx + e0 + j) : -1;
      pk[k] = j;
      if (Part && base >= 0 && j < n) {
        const uint32_t w = (uint32_t)u[k];
        u[k] = base + (int32_t)(w >> kPosBits);
        pk[k] = (int32_t)(w & ((1u << kPosBits) - 1));
      }
    }
    int32_t ra[kRowsPerLane], rb[kRowsPerLane], dv[kRowsPerLane];
    VT yo[kRowsPerLane];
#pragma unroll
    for (int q = 0; q < kRowsPerLane; ++q) {
      const int32_t v = v0 + t + q * kBlock;
      ra[q] = rb[q] = 0;
      dv[q] = 0;
      yo[q] = (VT)0;
      if (v < v1) {
        ra[q] = __builtin_nontemporal_load(off + v) - e0;
        rb[q] = __builtin_nontemporal_load(off + v + 1) - e0;
        if (!Part) {
          dv[q] = __builtin_nontemporal_load(c.outdeg + v);
          yo[q] = __builtin_nontemporal_load(yin + v);
        }
      }
    }
    VT x[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) x[k] = u[k] >= 0 ? xs[u[k]] : (VT)0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int j = t + k * kBlock;
      if (j < n) vals[pk[k]] = x[k];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRowsPerLane; ++q) {
      const int32_t v = v0 + t + q * kBlock;
      const bool mine = v < v1;
      const bool mid = mine && (rb[q] - ra[q]) > c.mid_deg;
      if (mine && !mid) {
        VT s = (VT)0;
        for (int32_t j = ra[q]; j < rb[q]; ++j) s += vals[j];
        if (Part)
          store_partial(&c.part[v], s);
        else
          epilogue<VT>(v, (double)s, c.c0, c.alpha, dv[q], yo[q], yout, a);
      }
      unsigned long long m = __ballot(mid);
      while (m) {
        const int src = __ffsll((long long)m) - 1;
        m &= m - 1;
        const int32_t wa = __shfl(ra[q], src, 64), wb = __shfl(rb[q], src, 64);
        VT s = (VT)0;
        for (int32_t j = wa + lane; j < wb; j += 64) s += vals[j];
        s = wave_sum(s);
        if (lane == src) {
          if (Part)
            store_partial(&c.part[v], s);
          else
            epilogue<VT>(v, (double)s, c.c0, c.alpha, dv[q], yo[q], yout, a);
        }
      }
    }
    __syncthreads();
  } else {
    // ---- one segment [e0, e1) (at most kSeg entries) of a long row, summed by the block
    const int32_t v = d.x, slot = d.w;
    VT s = (VT)0;
    for (int32_t cc = e0; cc < e1; cc += kSpan) {
      const int32_t n = min(kSpan, e1 - cc);
      int32_t u[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int j = t + k * kBlock;
        u[k] = j < n ? __builtin_nontemporal_load(idx + cc + j) : -1;
      }
      VT x[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) x[k] = u[k] >= 0 ? xs[u[k]] : (VT)0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) s += x[k];
    }
    const double seg = block_sum((double)s, red);
    if (t == 0) {
      if (Part)
        c.part[v] = (VT)seg;  // not reached: pairs are never longer than a tile window
      else if (slot < 0)
        epilogue<VT>(v, seg, c.c0, c.alpha, c.outdeg[v], yin[v], yout, a);
      else
        c.hpart[slot] = seg;
    }
  }
}

}  // namespace prpull
