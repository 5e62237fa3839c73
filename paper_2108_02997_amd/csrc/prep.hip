// prep.hip -- per-graph work partition (degree binning) on the device.
//
// The pull update needs, for every vertex v, the sum over v's in-edges (paper, section 2).
// Rows are cut into tiles for the gather kernel:
//   * a run of consecutive rows whose first entry falls in one window of kTile CSR entries and
//     whose ids fall in one window of kRows rows is one tile: its entries (fewer than 2*kTile)
//     are staged through LDS with coalesced index loads; rows of in-degree <= kMidDeg are then
//     summed by one lane each, longer ones by a whole wave64;
//   * a row with more than kTile entries (a hub) gets its own tiles, one per kTile-entry
//     segment, combined in a fixed order by the last segment to finish.
// The tile starts are found by a data-parallel rule evaluated per row, so the partition is a
// flag-and-scan: count descriptors per row, exclusive scan, write descriptors.
#include "internal.h"

namespace prpull {

constexpr int kScanChunk = 4096;               // rows per scan block
constexpr int kScanPerLane = kScanChunk / kBlock;  // 16 consecutive rows per lane

int64_t max_desc(int64_t N, int64_t E) { return 4 * (E / kTile + 1) + N / kRows + 8; }
int64_t max_slots(int64_t N, int64_t E) {
  (void)N;
  return 2 * (E / kTile) + 2;
}

static int64_t scan_blocks(int64_t N) { return (N + kScanChunk - 1) / kScanChunk; }
int64_t scan_block_count(int64_t N) { return scan_blocks(N); }

size_t prep_bytes(int64_t N, int64_t E) {
  size_t b = align_up(sizeof(PrepHeader), 256);
  b += align_up((size_t)(max_desc(N, E) + 1) * sizeof(int4), 256);
  b += align_up((size_t)(scan_blocks(N) + 1) * sizeof(unsigned long long), 256);
  return b;
}

// Number of descriptors starting at row v (high 32 bits) and hub segment slots of v (low 32).
__device__ __forceinline__ unsigned long long row_code(const int32_t *__restrict__ off, int32_t v) {
  const int32_t a = off[v], b = off[v + 1];
  const int32_t deg = b - a;
  const bool hub = deg > kTile;
  bool start = true;
  if (v > 0) {
    const int32_t pa = off[v - 1];
    const bool prev_hub = (a - pa) > kTile;
    start = hub || prev_hub || (a / kTile != pa / kTile) || (v / kRows != (v - 1) / kRows);
  }
  if (!start) return 0ull;
  if (hub) {
    const unsigned long long ns = (unsigned long long)((deg + kTile - 1) / kTile);
    return (ns << 32) | ns;
  }
  return 1ull << 32;
}

__device__ __forceinline__ unsigned long long block_exclusive_scan(unsigned long long x,
                                                                   unsigned long long *lds,
                                                                   unsigned long long *total) {
  const int t = threadIdx.x;
  lds[t] = x;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    unsigned long long y = t >= o ? lds[t - o] : 0ull;
    __syncthreads();
    lds[t] += y;
    __syncthreads();
  }
  const unsigned long long incl = lds[t];
  *total = lds[kBlock - 1];
  __syncthreads();
  return incl - x;
}

__global__ __launch_bounds__(kBlock) void k_prep_reduce(const int32_t *__restrict__ off, int32_t N,
                                                        unsigned long long *__restrict__ bsum) {
  __shared__ unsigned long long lds[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPerLane;
  unsigned long long s = 0;
  for (int k = 0; k < kScanPerLane; ++k) {
    const int64_t v = base + k;
    if (v < N) s += row_code(off, (int32_t)v);
  }
  unsigned long long tot;
  block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One block: exclusive scan of the block sums in place; total in bsum[nb]; writes the sentinel.
__global__ __launch_bounds__(kBlock) void k_prep_top(unsigned long long *__restrict__ bsum, int64_t nb,
                                                     int4 *__restrict__ desc, int32_t N) {
  __shared__ unsigned long long lds[kBlock];
  unsigned long long carry = 0;
  for (int64_t c = 0; c < nb; c += kBlock) {
    const int64_t i = c + threadIdx.x;
    const unsigned long long x = i < nb ? bsum[i] : 0ull;
    unsigned long long tot;
    const unsigned long long ex = block_exclusive_scan(x, lds, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    bsum[nb] = carry;
    desc[carry >> 32] = make_int4(N, 0, -1, 0);
  }
}

__global__ __launch_bounds__(kBlock) void k_prep_write(const int32_t *__restrict__ off, int32_t N,
                                                       const unsigned long long *__restrict__ bsum,
                                                       int4 *__restrict__ desc) {
  __shared__ unsigned long long lds[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPerLane;
  unsigned long long s = 0;
  for (int k = 0; k < kScanPerLane; ++k) {
    const int64_t v = base + k;
    if (v < N) s += row_code(off, (int32_t)v);
  }
  unsigned long long tot;
  unsigned long long pos = bsum[blockIdx.x] + block_exclusive_scan(s, lds, &tot);
  for (int k = 0; k < kScanPerLane; ++k) {
    const int64_t v = base + k;
    if (v >= N) break;
    const unsigned long long c = row_code(off, (int32_t)v);
    if (c == 0) continue;
    const int32_t p = (int32_t)(pos >> 32);
    const int32_t q = (int32_t)(pos & 0xffffffffull);
    const int32_t nd = (int32_t)(c >> 32);
    const int32_t ns = (int32_t)(c & 0xffffffffull);
    if (ns > 0) {
      for (int32_t s2 = 0; s2 < ns; ++s2) desc[p + s2] = make_int4((int32_t)v, ns, s2, q);
    } else {
      desc[p] = make_int4((int32_t)v, 0, -1, 0);
    }
    (void)nd;
    pos += c;
  }
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, int64_t n, uint32_t v) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

// Runs the three partition kernels, then copies the packed total (descriptors << 32 | hub slots)
// to host_total (host memory) and synchronises the stream.
hipError_t launch_prepare(hipStream_t s, const int32_t *off, int64_t N, int4 *desc,
                           unsigned long long *bsum, unsigned long long *host_total) {
  const int64_t nb = scan_blocks(N);
  hipLaunchKernelGGL(k_prep_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, off, (int32_t)N, bsum);
  hipLaunchKernelGGL(k_prep_top, dim3(1), dim3(kBlock), 0, s, bsum, nb, desc, (int32_t)N);
  hipLaunchKernelGGL(k_prep_write, dim3((unsigned)nb), dim3(kBlock), 0, s, off, (int32_t)N, bsum, desc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host_total, bsum + nb, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace prpull
