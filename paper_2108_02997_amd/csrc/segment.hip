// segment.hip -- source-segmented layout of the in-edge CSR, a locality preprocessing for the
// pull gather (it reorders the additions of each row's sum of section 2 into per-segment
// partial sums; the terms summed are the same).
//
// Source ids are cut into segments of seg_len consecutive ids, sized so that one segment's slice
// of the iterate stays resident in an XCD's L2 while its entries are gathered.  A pair is a run
// of one row's entries whose sources lie in one segment, cut at row-relative multiples of
// kPairMax entries (so no pair needs more than one tile).  The update then runs in two steps:
//   per-segment step: over the pairs listed segment by segment (the pair CSR poff / sidx), each
//                     pair's entries are summed into partial[pair];
//   merge step      : every row sums its pairs' partials in segment order (the merge CSR
//                     moff / mpos) and runs the usual epilogue.
// Building it (once per graph):
//   1. F[j] = 1 where entry j starts a pair (first entry of its row, a new segment, or a
//      row-relative multiple of kPairMax); X = exclusive scan of F, so pair q (numbered in row
//      order) starts at the entry j with F[j] = 1 and X[j] = q, and P = X[E];
//   2. per pair (row order): its start, its segment (the sort key) and its number q;
//      moff[v] = X[off[v]] (a row's pairs in row order are consecutive);
//   3. a stable radix sort of the pairs by segment (hipCUB) gives perm[p] = q, the row-order
//      pair at segment-major position p; mpos[q] = p; pair lengths in segment-major order;
//   4. poff = exclusive scan of the lengths; every entry is copied to its place in sidx.
// After the pair CSR's tile partition is built (api.hip), every pair tile's entries are sorted by
// source and packed with their pair-order positions (launch_seg_tile_sort, below).
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace prpull {

constexpr int kSegCountBlocks = 1024;

int64_t seg_count_blocks() { return kSegCountBlocks; }

// Row of entry j: the largest v with off[v] <= j (0 <= j < off[N]).
__device__ __forceinline__ int32_t row_of(const int32_t *__restrict__ off, int32_t N, int32_t j) {
  int32_t lo = 0, hi = N - 1;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo + 1) >> 1);
    if (off[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int32_t pair_start(const int32_t *__restrict__ off, const int32_t *__restrict__ idx,
                                              int32_t N, int32_t seg_len, int32_t j) {
  const int32_t rel = j - off[row_of(off, N, j)];
  if (rel % kPairMax == 0) return 1;
  return idx[j] / seg_len != idx[j - 1] / seg_len ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_seg_count(const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ idx, int32_t N, int32_t E,
                                                      int32_t seg_len, unsigned long long *__restrict__ part) {
  __shared__ unsigned long long red[kWaves];
  unsigned long long n = 0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < E; j += (int64_t)gridDim.x * kBlock)
    n += (unsigned long long)pair_start(off, idx, N, seg_len, (int32_t)j);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < kWaves; ++w) s += red[w];
    part[blockIdx.x] = s;
  }
}

__global__ void k_seg_count_total(unsigned long long *part, int32_t nb) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    unsigned long long s = 0;
    for (int32_t b = 0; b < nb; ++b) s += part[b];
    part[nb] = s;
  }
}

hipError_t launch_seg_count(hipStream_t s, const int32_t *off, const int32_t *idx, int32_t N, int32_t E,
                            int32_t seg_len, unsigned long long *block_counts, unsigned long long *host_total) {
  hipLaunchKernelGGL(k_seg_count, dim3(kSegCountBlocks), dim3(kBlock), 0, s, off, idx, N, E, seg_len, block_counts);
  hipLaunchKernelGGL(k_seg_count_total, dim3(1), dim3(64), 0, s, block_counts, (int32_t)kSegCountBlocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host_total, block_counts + kSegCountBlocks, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                     s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// Step 1: F[j] for j < E, F[E] = 0.
__global__ __launch_bounds__(kBlock) void k_seg_flags(const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ idx, int32_t N, int32_t E,
                                                      int32_t seg_len, int32_t *__restrict__ F) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j <= E; j += (int64_t)gridDim.x * kBlock)
    F[j] = j < E ? pair_start(off, idx, N, seg_len, (int32_t)j) : 0;
}

// Step 2: per pair in row order; pstart[P] = E.
__global__ __launch_bounds__(kBlock) void k_seg_pairs(const int32_t *__restrict__ idx, const int32_t *__restrict__ F,
                                                      const int32_t *__restrict__ X, int32_t E, int32_t seg_len,
                                                      int32_t *__restrict__ pstart, int32_t *__restrict__ pseg,
                                                      int32_t *__restrict__ pq) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j <= E; j += (int64_t)gridDim.x * kBlock) {
    if (j == E) {
      pstart[X[E]] = E;
    } else if (F[j]) {
      const int32_t q = X[j];
      pstart[q] = (int32_t)j;
      pseg[q] = idx[j] / seg_len;
      pq[q] = q;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_seg_moff(const int32_t *__restrict__ off, const int32_t *__restrict__ X,
                                                     int32_t N, int32_t *__restrict__ moff) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v <= N; v += (int64_t)gridDim.x * kBlock)
    moff[v] = X[off[v]];
}

// Step 3: perm[p] = q -> mpos[q] = p, plen[p] = length of pair q; plen[P] = 0.
__global__ __launch_bounds__(kBlock) void k_seg_place(const int32_t *__restrict__ perm,
                                                      const int32_t *__restrict__ pstart, int32_t P,
                                                      int32_t *__restrict__ mpos, int32_t *__restrict__ plen) {
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p <= P; p += (int64_t)gridDim.x * kBlock) {
    if (p == P) {
      plen[P] = 0;
    } else {
      const int32_t q = perm[p];
      mpos[q] = (int32_t)p;
      plen[p] = pstart[q + 1] - pstart[q];
    }
  }
}

// Step 4: entry j of pair q (row order) goes to sidx[poff[mpos[q]] + j - pstart[q]].
__global__ __launch_bounds__(kBlock) void k_seg_scatter(const int32_t *__restrict__ idx,
                                                        const int32_t *__restrict__ X,
                                                        const int32_t *__restrict__ pstart,
                                                        const int32_t *__restrict__ mpos,
                                                        const int32_t *__restrict__ poff, int32_t E,
                                                        int32_t *__restrict__ sidx) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < E; j += (int64_t)gridDim.x * kBlock) {
    const int32_t q = X[j + 1] - 1;
    sidx[poff[mpos[q]] + ((int32_t)j - pstart[q])] = idx[j];
  }
}

static unsigned grid_n(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (unsigned)(g < 1 ? 1 : g > 16384 ? 16384 : g);
}

hipError_t seg_sort_temp_bytes(int64_t P, int key_bits, size_t *bytes) {
  *bytes = 0;
  return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const int32_t *)nullptr, (int32_t *)nullptr,
                                            (const int32_t *)nullptr, (int32_t *)nullptr, (int)(P > 0 ? P : 1), 0,
                                            key_bits, (hipStream_t)0);
}

hipError_t seg_scan_temp_bytes(int64_t n, size_t *bytes) {
  *bytes = 0;
  return hipcub::DeviceScan::ExclusiveSum(nullptr, *bytes, (const int32_t *)nullptr, (int32_t *)nullptr,
                                          (int)(n > 0 ? n : 1), (hipStream_t)0);
}

// ---- tile order (after the pair partition is built): every pair tile's entries sorted by source
// (hipCUB's segmented radix sort over the tiles, carrying each entry's pair-order position), then
// packed: a tile whose sources span fewer than 2^kRelBits ids keeps, per entry, the source less
// the tile's smallest source (high bits) and the entry's pair-order position (low kPosBits bits),
// and its descriptor's w holds that smallest source; any other tile keeps its pair order, w = -1.
static_assert(kSpan <= (1 << kPosBits), "tile positions fit the packed word");

__global__ __launch_bounds__(kBlock) void k_tile_offsets(const int4 *__restrict__ pdesc, int32_t ndesc,
                                                         int32_t *__restrict__ toff) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= ndesc; i += (int64_t)gridDim.x * kBlock)
    toff[i] = pdesc[i].y;
}

// Pair-order position of every entry within its tile (one workgroup per tile; tiles hold fewer
// than kSpan entries).
__global__ __launch_bounds__(kBlock) void k_tile_positions(const int32_t *__restrict__ toff, int32_t ndesc,
                                                           uint16_t *__restrict__ pos) {
  for (int32_t i = blockIdx.x; i < ndesc; i += gridDim.x) {
    const int32_t e0 = toff[i], e1 = toff[i + 1];
    for (int32_t j = e0 + threadIdx.x; j < e1; j += kBlock) pos[j] = (uint16_t)(j - e0);
  }
}

// keys / pos: the tiles sorted by source with their positions; writes sidx and pdesc[i].w.
__global__ __launch_bounds__(kBlock) void k_tile_pack(const int32_t *__restrict__ toff, int32_t ndesc,
                                                      const int32_t *__restrict__ keys,
                                                      const uint16_t *__restrict__ pos, int32_t *__restrict__ sidx,
                                                      int4 *__restrict__ pdesc) {
  for (int32_t i = blockIdx.x; i < ndesc; i += gridDim.x) {
    const int32_t e0 = toff[i], e1 = toff[i + 1];
    if (e1 <= e0) {
      if (threadIdx.x == 0) pdesc[i].w = -1;
      continue;
    }
    const int32_t lo = keys[e0];
    const bool packed = keys[e1 - 1] - lo < (1 << kRelBits);
    for (int32_t j = e0 + threadIdx.x; j < e1; j += kBlock) {
      if (packed)
        sidx[j] = (int32_t)(((uint32_t)(keys[j] - lo) << kPosBits) | (uint32_t)pos[j]);
      else
        sidx[e0 + pos[j]] = keys[j];
    }
    if (threadIdx.x == 0) pdesc[i].w = packed ? lo : -1;
  }
}

hipError_t seg_tile_sort_temp_bytes(int64_t E, int64_t tiles, int key_bits, size_t *bytes) {
  *bytes = 0;
  return hipcub::DeviceSegmentedRadixSort::SortPairs(
      nullptr, *bytes, (const int32_t *)nullptr, (int32_t *)nullptr, (const uint16_t *)nullptr, (uint16_t *)nullptr,
      (int)(E > 0 ? E : 1), (int)(tiles > 0 ? tiles : 1), (const int32_t *)nullptr, (const int32_t *)nullptr, 0,
      key_bits, (hipStream_t)0);
}

size_t seg_tile_sort_scratch(int64_t E, int64_t tiles, size_t sort_bytes) {
  return align_up(4 * (size_t)(tiles + 1), 256) + 2 * align_up(2 * (size_t)E, 256) + align_up(sort_bytes, 256);
}

// The sorted keys pass through the construction scratch temp (E + 1 values); tile offsets,
// positions and the sort's storage sit in the scratch at sl.tsort_off.
hipError_t launch_seg_tile_sort(hipStream_t s, int4 *pdesc, int32_t ndesc, int32_t E, int key_bits, char *base,
                                const SegLayout &sl) {
  int32_t *sidx = (int32_t *)(base + sl.sidx_off);
  int32_t *keys = (int32_t *)(base + sl.temp_off);
  char *t = base + sl.tsort_off;
  int32_t *toff = (int32_t *)t;
  t += align_up(4 * (size_t)(ndesc + 1), 256);
  uint16_t *pos_in = (uint16_t *)t;
  t += align_up(2 * (size_t)E, 256);
  uint16_t *pos = (uint16_t *)t;
  t += align_up(2 * (size_t)E, 256);
  size_t bytes = 0;
  hipError_t e = seg_tile_sort_temp_bytes(E, ndesc, key_bits, &bytes);
  if (e != hipSuccess) return e;
  if ((int64_t)(t - base) + (int64_t)bytes > sl.tsort_off + sl.tsort_bytes) return hipErrorInvalidValue;
  const unsigned tiles_grid = (unsigned)std::min<int32_t>(std::max<int32_t>(ndesc, 1), 16384);
  hipLaunchKernelGGL(k_tile_offsets, dim3(grid_n((int64_t)ndesc + 1)), dim3(kBlock), 0, s, pdesc, ndesc, toff);
  hipLaunchKernelGGL(k_tile_positions, dim3(tiles_grid), dim3(kBlock), 0, s, toff, ndesc, pos_in);
  e = hipcub::DeviceSegmentedRadixSort::SortPairs((void *)t, bytes, sidx, keys, pos_in, pos, (int)E, (int)ndesc, toff,
                                                  toff + 1, 0, key_bits, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_pack, dim3(tiles_grid), dim3(kBlock), 0, s, toff, ndesc, keys, pos, sidx, pdesc);
  return hipGetLastError();
}

// The whole build into the buffer at `base` (layout sl, sizes checked by the caller; P > 0).
// Construction scratch: F aliases sidx (E + 1 values), the sort's inputs alias part (2P values);
// X, pstart, the sort keys' output (later the pair lengths), perm and hipCUB's storage sit at
// temp_off.
hipError_t launch_seg_build(hipStream_t s, const int32_t *off, const int32_t *idx, int32_t N, int32_t E,
                            int32_t seg_len, int key_bits, int64_t P, char *base, const SegLayout &sl) {
  int32_t *poff = (int32_t *)(base + sl.poff_off);
  int32_t *moff = (int32_t *)(base + sl.moff_off);
  int32_t *mpos = (int32_t *)(base + sl.mpos_off);
  int32_t *sidx = (int32_t *)(base + sl.sidx_off);
  int32_t *F = sidx;
  int32_t *pseg = (int32_t *)(base + sl.part_off);
  int32_t *pq = pseg + P;
  char *t = base + sl.temp_off;
  int32_t *X = (int32_t *)t;
  t += align_up(4 * (size_t)(E + 1), 256);
  int32_t *pstart = (int32_t *)t;
  t += align_up(4 * (size_t)(P + 1), 256);
  int32_t *kout = (int32_t *)t;  // sort keys out, then the pair lengths (P + 1 values)
  t += align_up(4 * (size_t)(P + 1), 256);
  int32_t *perm = (int32_t *)t;
  void *cub = (void *)(base + sl.cub_off);
  size_t sort_b = 0, scan_e = 0, scan_p = 0;
  hipError_t e = seg_sort_temp_bytes(P, key_bits, &sort_b);
  if (e == hipSuccess) e = seg_scan_temp_bytes(E + 1, &scan_e);
  if (e == hipSuccess) e = seg_scan_temp_bytes(P + 1, &scan_p);
  if (e != hipSuccess) return e;

  hipLaunchKernelGGL(k_seg_flags, dim3(grid_n(E + 1)), dim3(kBlock), 0, s, off, idx, N, E, seg_len, F);
  e = hipcub::DeviceScan::ExclusiveSum(cub, scan_e, F, X, (int)(E + 1), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_pairs, dim3(grid_n(E + 1)), dim3(kBlock), 0, s, idx, F, X, E, seg_len, pstart, pseg, pq);
  hipLaunchKernelGGL(k_seg_moff, dim3(grid_n((int64_t)N + 1)), dim3(kBlock), 0, s, off, X, N, moff);
  e = hipcub::DeviceRadixSort::SortPairs(cub, sort_b, pseg, kout, pq, perm, (int)P, 0, key_bits, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_place, dim3(grid_n(P + 1)), dim3(kBlock), 0, s, perm, pstart, (int32_t)P, mpos, kout);
  e = hipcub::DeviceScan::ExclusiveSum(cub, scan_p, kout, poff, (int)(P + 1), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_scatter, dim3(grid_n(E)), dim3(kBlock), 0, s, idx, X, pstart, mpos, poff, E, sidx);
  return hipGetLastError();
}

}  // namespace prpull
