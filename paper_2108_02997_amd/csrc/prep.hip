// prep.hip -- per-graph work partition (degree binning) on the device.
//
// The pull update needs, for every vertex v, the sum over v's in-edges (paper, section 2).
// Rows are cut into tiles for the gather kernel:
//   * a run of consecutive rows whose first entry falls in one window of kTile CSR entries and
//     whose ids fall in one window of kRows rows is one tile: its entries (fewer than 2*kTile)
//     are staged through LDS with coalesced index loads; rows of in-degree <= kMidDeg are then
//     summed by one lane each, longer ones by a whole wave64;
//   * a row with more than kTile entries (a long row) gets tiles of its own, one per segment of
//     at most kSeg entries, each summed by one workgroup.  A long row of one segment finishes in
//     that workgroup; a row of several segments (a hub) leaves one partial sum per segment,
//     combined in segment order by the finishing kernel, which walks the hub table.
// Tile starts follow a rule evaluated per row, so the partition is a flag-and-scan: count
// descriptors, segment slots and hubs per row, exclusive scan, write descriptors.
#include "internal.h"

namespace prpull {

constexpr int kScanChunk = 4096;                   // rows per scan block
constexpr int kScanPerLane = kScanChunk / kBlock;  // 16 consecutive rows per lane

int64_t max_desc(int64_t N, int64_t E, int tile, int rows) { return 4 * (E / tile + 1) + N / rows + 8; }
int64_t max_slots(int64_t N, int64_t E) {
  (void)N;
  return 2 * (E / kSeg) + 2;
}
int64_t max_hubs(int64_t N, int64_t E) {
  (void)N;
  return E / kSeg + 1;
}

static int64_t scan_blocks(int64_t N) { return (N + kScanChunk - 1) / kScanChunk; }
int64_t scan_block_count(int64_t N) { return scan_blocks(N); }

// Layout: header | partition A (descriptors, hubs) | partition B (descriptors, hubs) | scan scratch.
// Each partition is sized for the smallest window it may be given (the autotuner's candidates).
size_t prep_bytes(int64_t N, int64_t E) {
  size_t b = align_up(sizeof(PrepHeader), 256);
  for (int i = 0; i < 2; ++i) {
    b += align_up((size_t)(max_desc(N, E, kMinPartTile[i], kMinPartRows[i]) + 1) * sizeof(int4), 256);
    b += align_up((size_t)max_hubs(N, E) * sizeof(int4), 256);
  }
  b += align_up((size_t)(scan_blocks(N) + 1) * 2 * sizeof(unsigned long long), 256);
  return b;
}

bool valid_window(int part, int tile, int rows) {
  if (part == 0) return (tile == 1024 && rows == 512) || (tile == 512 && rows == 256) || (tile == 256 && rows == 128);
  return (tile == 256 && rows == 128) || (tile == 128 && rows == 64);
}

// Per-row counts: a = descriptors starting at row v, b = (segment slots << 32) | hubs.
struct Code {
  unsigned long long a, b;
};
__device__ __forceinline__ Code operator+(Code x, Code y) { return Code{x.a + y.a, x.b + y.b}; }
__device__ __forceinline__ Code operator-(Code x, Code y) { return Code{x.a - y.a, x.b - y.b}; }

template <int TILE, int ROWS>
__device__ __forceinline__ Code row_code(const int32_t *__restrict__ off, int32_t v) {
  const int32_t a = off[v], b = off[v + 1];
  const int32_t deg = b - a;
  const bool lng = deg > TILE;
  bool start = true;
  if (v > 0) {
    const int32_t pa = off[v - 1];
    const bool prev_long = (a - pa) > TILE;
    start = lng || prev_long || (a / TILE != pa / TILE) || (v / ROWS != (v - 1) / ROWS);
  }
  if (!start) return Code{0ull, 0ull};
  if (lng) {
    const unsigned long long ns = (unsigned long long)((deg + kSeg - 1) / kSeg);
    if (ns == 1) return Code{1ull, 0ull};
    return Code{ns, (ns << 32) | 1ull};
  }
  return Code{1ull, 0ull};
}

__device__ __forceinline__ Code block_exclusive_scan(Code x, Code *lds, Code *total) {
  const int t = threadIdx.x;
  lds[t] = x;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const Code y = t >= o ? lds[t - o] : Code{0ull, 0ull};
    __syncthreads();
    lds[t] = lds[t] + y;
    __syncthreads();
  }
  const Code incl = lds[t];
  *total = lds[kBlock - 1];
  __syncthreads();
  return incl - x;
}

template <int TILE, int ROWS>
__global__ __launch_bounds__(kBlock) void k_prep_reduce(const int32_t *__restrict__ off, int32_t N,
                                                        Code *__restrict__ bsum) {
  __shared__ Code lds[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPerLane;
  Code s{0ull, 0ull};
  for (int k = 0; k < kScanPerLane; ++k) {
    const int64_t v = base + k;
    if (v < N) s = s + row_code<TILE, ROWS>(off, (int32_t)v);
  }
  Code tot;
  block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One block: exclusive scan of the block sums in place; total in bsum[nb]; writes the sentinel.
__global__ __launch_bounds__(kBlock) void k_prep_top(Code *__restrict__ bsum, int64_t nb, int4 *__restrict__ desc,
                                                     const int32_t *__restrict__ off, int32_t N) {
  __shared__ Code lds[kBlock];
  Code carry{0ull, 0ull};
  for (int64_t c = 0; c < nb; c += kBlock) {
    const int64_t i = c + threadIdx.x;
    const Code x = i < nb ? bsum[i] : Code{0ull, 0ull};
    Code tot;
    const Code ex = block_exclusive_scan(x, lds, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry = carry + tot;
  }
  if (threadIdx.x == 0) {
    bsum[nb] = carry;
    desc[carry.a] = make_int4(N, off[N], -1, -1);
  }
}

template <int TILE, int ROWS>
__global__ __launch_bounds__(kBlock) void k_prep_write(const int32_t *__restrict__ off, int32_t N,
                                                       const Code *__restrict__ bsum, int4 *__restrict__ desc,
                                                       int4 *__restrict__ hubs) {
  __shared__ Code lds[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPerLane;
  Code s{0ull, 0ull};
  for (int k = 0; k < kScanPerLane; ++k) {
    const int64_t v = base + k;
    if (v < N) s = s + row_code<TILE, ROWS>(off, (int32_t)v);
  }
  Code tot;
  Code pos = bsum[blockIdx.x] + block_exclusive_scan(s, lds, &tot);
  for (int k = 0; k < kScanPerLane; ++k) {
    const int64_t v = base + k;
    if (v >= N) break;
    const Code c = row_code<TILE, ROWS>(off, (int32_t)v);
    if (c.a == 0) continue;
    const int32_t p = (int32_t)pos.a;
    const int32_t slot = (int32_t)(pos.b >> 32);
    const int32_t hub = (int32_t)(pos.b & 0xffffffffull);
    const int32_t ev = off[v];
    const int32_t deg = off[v + 1] - ev;
    if (deg > TILE) {
      const int32_t ns = (int32_t)c.a;
      if (ns == 1) {
        desc[p] = make_int4((int32_t)v, ev, 0, -1);
      } else {
        for (int32_t sg = 0; sg < ns; ++sg) desc[p + sg] = make_int4((int32_t)v, ev + sg * kSeg, sg, slot + sg);
        hubs[hub] = make_int4((int32_t)v, ns, slot, 0);
      }
    } else {
      desc[p] = make_int4((int32_t)v, ev, -1, -1);
    }
    pos = pos + c;
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

// Runs the three partition kernels of partition `part` (0: update tiles, 1: batch tiles), copies
// the totals {descriptors, slots << 32 | hubs} to host_total (host memory, 2 words) and
// synchronises the stream.
template <int TILE, int ROWS>
static hipError_t prepare_part(hipStream_t s, const int32_t *off, int64_t N, int4 *desc, int4 *hubs, Code *bsum) {
  const int64_t nb = scan_blocks(N);
  hipLaunchKernelGGL((k_prep_reduce<TILE, ROWS>), dim3((unsigned)nb), dim3(kBlock), 0, s, off, (int32_t)N, bsum);
  hipLaunchKernelGGL(k_prep_top, dim3(1), dim3(kBlock), 0, s, bsum, nb, desc, off, (int32_t)N);
  hipLaunchKernelGGL((k_prep_write<TILE, ROWS>), dim3((unsigned)nb), dim3(kBlock), 0, s, off, (int32_t)N, bsum, desc,
                     hubs);
  return hipGetLastError();
}

hipError_t launch_prepare(hipStream_t s, int tile, int rows, const int32_t *off, int64_t N, int4 *desc, int4 *hubs,
                          void *scan, unsigned long long *host_total) {
  Code *bsum = (Code *)scan;
  hipError_t e;
  if (tile == 1024 && rows == 512)
    e = prepare_part<1024, 512>(s, off, N, desc, hubs, bsum);
  else if (tile == 512 && rows == 256)
    e = prepare_part<512, 256>(s, off, N, desc, hubs, bsum);
  else if (tile == 256 && rows == 128)
    e = prepare_part<256, 128>(s, off, N, desc, hubs, bsum);
  else if (tile == 128 && rows == 64)
    e = prepare_part<128, 64>(s, off, N, desc, hubs, bsum);
  else if (tile == kPairTile && rows == kRows)  // the pair partition of the segmented layout
    e = prepare_part<kPairTile, kRows>(s, off, N, desc, hubs, bsum);
  else
    return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host_total, bsum + scan_blocks(N), sizeof(Code), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace prpull
