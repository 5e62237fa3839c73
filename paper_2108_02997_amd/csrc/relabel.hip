// relabel.hip -- degree ordering of the vertices, a locality preprocessing for the pull gather
// (not part of the paper's method: it renames vertices, the ranks it computes are the same up to
// the renaming).  perm[v] = new id of v: vertices by decreasing out-degree, ties by id, so the most
// cited sources get consecutive ids and their contributions share cache lines.  Row perm[v] of the
// relabelled in-CSR holds v's in-edges, each source u renamed perm[u], in ascending order.
//
// Steps: a stable radix sort of (out-degree, id) pairs in descending key order (hipCUB), the
// inverse permutation and the new row lengths, an exclusive scan of the lengths (hipCUB), one wave
// per new row renaming its entries and sorting rows of at most 64 entries in registers, and a
// segmented radix sort (hipCUB) of the longer rows.
#include <hipcub/hipcub.hpp>

#include "relabel.h"

namespace prpull {

__global__ __launch_bounds__(kBlock) void k_relabel_keys(const int32_t *__restrict__ outdeg, int32_t N,
                                                         uint32_t *__restrict__ key, int32_t *__restrict__ val) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock) {
    key[v] = (uint32_t)outdeg[v];
    val[v] = (int32_t)v;
  }
}

// order[k] = old id at new position k  ->  perm, new row lengths (len[N] = 0 closes the scan) and
// the new out-degrees.
__global__ __launch_bounds__(kBlock) void k_relabel_perm(const int32_t *__restrict__ order,
                                                         const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ outdeg, int32_t N,
                                                         int32_t *__restrict__ perm, int32_t *__restrict__ len,
                                                         int32_t *__restrict__ new_outdeg) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k <= N; k += (int64_t)gridDim.x * kBlock) {
    if (k == N) {
      len[N] = 0;
      continue;
    }
    const int32_t v = order[k];
    perm[v] = (int32_t)k;
    len[k] = off[v + 1] - off[v];
    new_outdeg[k] = outdeg[v];
  }
}

// Ascending bitonic sort of one value per lane across a wave.
__device__ __forceinline__ int32_t wave_sort_asc(int32_t x, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int32_t o = __shfl_xor(x, j, 64);
      const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
      x = keep_min ? min(x, o) : max(x, o);
    }
  }
  return x;
}

// One wave per new row: the entries of old row order[k], sources renamed and sorted ascending in
// chunks of 64 (a whole row when it has at most 64 entries; longer rows are sorted whole
// afterwards), so that a tile's gathers walk the renamed sources in address order.
__global__ __launch_bounds__(kBlock) void k_relabel_rows(const int32_t *__restrict__ order,
                                                         const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ idx,
                                                         const int32_t *__restrict__ perm,
                                                         const int32_t *__restrict__ new_off, int32_t N,
                                                         int32_t *__restrict__ new_idx) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * kWaves;
  for (int64_t k = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); k < N; k += waves) {
    const int32_t v = order[k];
    const int32_t a = off[v], n = off[v + 1] - a, b = new_off[k];
    for (int32_t c = 0; c < n; c += 64) {
      const int32_t j = c + lane;
      int32_t x = j < n ? perm[idx[a + j]] : INT32_MAX;
      x = wave_sort_asc(x, lane);
      if (j < n) new_idx[b + j] = x;
    }
  }
}

// Rows of more than 64 entries: their [begin, end) in the new CSR, listed for a segmented sort (the
// order of the list does not matter: every segment is sorted on its own).
__global__ __launch_bounds__(kBlock) void k_relabel_long_rows(const int32_t *__restrict__ new_off, int32_t N,
                                                              int32_t *__restrict__ seg_begin,
                                                              int32_t *__restrict__ seg_end,
                                                              uint32_t *__restrict__ count) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < N; k += (int64_t)gridDim.x * kBlock) {
    const int32_t a = new_off[k], b = new_off[k + 1];
    if (b - a > 64) {
      const uint32_t i = atomicAdd(count, 1u);
      seg_begin[i] = a;
      seg_end[i] = b;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_unpermute(const int32_t *__restrict__ perm, int32_t N,
                                                      const double *__restrict__ in, double *__restrict__ out) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock)
    out[v] = in[perm[v]];
}

static unsigned grid_of(int64_t n, int64_t per_block) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g > 8192 ? 8192 : g);
}

// Workspace: keys[2][N] u32, vals[2][N] i32, len[N+1] i32, seg_begin[N], seg_end[N] i32, a
// counter, a copy of the new indices [E] i32, then the hipCUB temporary storage.
static size_t relabel_arrays(int64_t N, int64_t E) {
  return align_up(4 * (size_t)N, 256) * 6 + align_up(4 * (size_t)(N + 1), 256) + 256 +
         align_up(4 * (size_t)(E > 0 ? E : 1), 256);
}

hipError_t relabel_temp_bytes(int64_t N, int64_t E, size_t *bytes) {
  size_t a = 0, b = 0, c = 0;
  hipcub::DoubleBuffer<uint32_t> k(nullptr, nullptr);
  hipcub::DoubleBuffer<int32_t> v(nullptr, nullptr);
  hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, a, k, v, (int)N, 0, 32, (hipStream_t)0);
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(nullptr, b, (const int32_t *)nullptr, (int32_t *)nullptr, (int)(N + 1),
                                       (hipStream_t)0);
  if (e != hipSuccess) return e;
  hipcub::DoubleBuffer<int32_t> r(nullptr, nullptr);
  e = hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, c, r, (int)(E > 0 ? E : 1), (int)N, (const int32_t *)nullptr,
                                                 (const int32_t *)nullptr, 0, 32, (hipStream_t)0);
  if (e != hipSuccess) return e;
  const size_t t = a > b ? (a > c ? a : c) : (b > c ? b : c);
  *bytes = relabel_arrays(N, E) + align_up(t, 256);
  return hipSuccess;
}

hipError_t launch_relabel(hipStream_t s, const int32_t *off, const int32_t *idx, const int32_t *outdeg, int32_t N,
                          int32_t E, int32_t *perm, int32_t *new_off, int32_t *new_idx, int32_t *new_outdeg,
                          void *ws, size_t ws_bytes, uint32_t *host_count) {
  char *p = (char *)ws;
  const size_t an = align_up(4 * (size_t)N, 256);
  uint32_t *k0 = (uint32_t *)p, *k1 = (uint32_t *)(p + an);
  int32_t *v0 = (int32_t *)(p + 2 * an), *v1 = (int32_t *)(p + 3 * an);
  int32_t *seg_begin = (int32_t *)(p + 4 * an), *seg_end = (int32_t *)(p + 5 * an);
  int32_t *len = (int32_t *)(p + 6 * an);
  uint32_t *count = (uint32_t *)(p + 6 * an + align_up(4 * (size_t)(N + 1), 256));
  int32_t *idx_copy = (int32_t *)((char *)count + 256);
  void *temp = p + relabel_arrays(N, E);
  const size_t temp_cap = ws_bytes - relabel_arrays(N, E);
  size_t temp_bytes = temp_cap;
  hipLaunchKernelGGL(k_relabel_keys, dim3(grid_of(N, kBlock)), dim3(kBlock), 0, s, outdeg, N, k0, v0);
  hipcub::DoubleBuffer<uint32_t> keys(k0, k1);
  hipcub::DoubleBuffer<int32_t> vals(v0, v1);
  hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(temp, temp_bytes, keys, vals, (int)N, 0, 32, s);
  if (e != hipSuccess) return e;
  const int32_t *order = vals.Current();
  hipLaunchKernelGGL(k_relabel_perm, dim3(grid_of((int64_t)N + 1, kBlock)), dim3(kBlock), 0, s, order, off, outdeg,
                     N, perm, len, new_outdeg);
  temp_bytes = temp_cap;
  e = hipcub::DeviceScan::ExclusiveSum(temp, temp_bytes, (const int32_t *)len, new_off, (int)(N + 1), s);
  if (e != hipSuccess) return e;
  if (E == 0) return hipGetLastError();
  hipLaunchKernelGGL(k_relabel_rows, dim3(grid_of(N, kWaves)), dim3(kBlock), 0, s, order, off, idx, perm, new_off, N,
                     new_idx);
  // rows longer than one wave: sorted whole by a segmented radix sort
  e = launch_fill_u32(s, count, 1, 0u);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_relabel_long_rows, dim3(grid_of(N, kBlock)), dim3(kBlock), 0, s, (const int32_t *)new_off, N,
                     seg_begin, seg_end, count);
  e = hipMemcpyAsync(host_count, count, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const uint32_t nseg = *host_count;
  if (nseg == 0) return hipSuccess;
  e = hipMemcpyAsync(idx_copy, new_idx, 4 * (size_t)E, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  // both buffers hold every entry; the sort touches only the listed segments
  hipcub::DoubleBuffer<int32_t> rows(new_idx, idx_copy);
  temp_bytes = temp_cap;
  e = hipcub::DeviceSegmentedRadixSort::SortKeys(temp, temp_bytes, rows, (int)E, (int)nseg,
                                                 (const int32_t *)seg_begin, (const int32_t *)seg_end, 0, 32, s);
  if (e != hipSuccess) return e;
  if (rows.Current() != new_idx) {
    e = hipMemcpyAsync(new_idx, rows.Current(), 4 * (size_t)E, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_unpermute(hipStream_t s, const int32_t *perm, int32_t N, const double *in, double *out) {
  hipLaunchKernelGGL(k_unpermute, dim3(grid_of(N, kBlock)), dim3(kBlock), 0, s, perm, N, in, out);
  return hipGetLastError();
}

}  // namespace prpull
