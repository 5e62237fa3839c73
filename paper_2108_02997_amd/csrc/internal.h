// internal.h -- shared definitions of the gfx950 pull-PageRank library (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace prpull {

// ---------------------------------------------------------------- tiling constants
// Block shape: 256 lanes = 4 wave64.
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
// A tile covers consecutive rows whose first CSR entry falls in one window of kTile entries
// and whose row ids fall in one window of kRows rows; rows longer than kTile are hubs and are
// cut into segments of kTile entries.  A tile therefore spans fewer than 2*kTile entries.
constexpr int kTile = 1024;
constexpr int kRows = 512;
constexpr int kSpan = 2 * kTile;
constexpr int kRowsPerLane = kRows / kBlock;  // 2
// Rows with in-degree above kMidDeg (and at most kTile) are summed by a whole wave.
constexpr int kMidDeg = 32;
// Upper bound of persistent-style grid (blocks loop over tiles).
constexpr int kMaxGrid = 4096;

// ---------------------------------------------------------------- prep layout
// Tile descriptor: x = first row, y = number of segments (hub) or 0 (tile of rows),
// z = segment index (hub) or -1, w = first partial slot of the hub.  Tile i ends where
// tile i+1 starts; a sentinel with x = N follows the last tile.
struct PrepHeader {
  int32_t magic;
  int32_t version;
  int64_t N;
  int64_t E;
  int32_t tile, rows, ndesc, nslots;
  int64_t desc_off;   // byte offset of the descriptors inside the prep buffer
  int64_t scan_off;   // byte offset of the scan scratch
  int64_t reserved[3];
};
constexpr int32_t kPrepMagic = 0x50525031;  // "PRP1"

size_t prep_bytes(int64_t N, int64_t E);
int64_t max_desc(int64_t N, int64_t E);
int64_t max_slots(int64_t N, int64_t E);

// ---------------------------------------------------------------- solve state (device)
struct alignas(64) SolveState {
  double c0;          // teleport term for the next update
  double err[3];      // L1, L2, Linf of the last update
  double prev_l1;     // L1 of the update before (float32 stagnation test)
  int32_t iter;       // updates performed so far (all phases)
  int32_t stop;       // 1: the kernels of the running phase are no-ops
  int32_t done;       // 1: the whole solve is finished
  int32_t converged;  // 1: an update met tau in the convergence norm
  int32_t phase_iter; // updates performed in the running phase
  int32_t met32;      // the float32 phase met tau
  uint32_t ticket;    // last-block counter of the iteration kernel
  uint32_t ticket2;   // last-block counter of init/convert kernels
  int32_t pad[4];
};

// Kernel parameters of one update (passed by value).
struct IterParams {
  const int32_t *off;
  const int32_t *idx;
  const int32_t *outdeg;
  const int4 *desc;
  int32_t ndesc;
  int32_t N;
  const void *y_in;
  void *y_out;
  double alpha;
  double tau;
  int32_t norm;
  int32_t max_iter;
  int32_t phase;       // 0: float64 solve, 1: float32 phase of a mixed solve, 2: float64 phase
  int32_t pad;
  SolveState *st;
  double *bpart;       // [gridDim.x][4] block partials: L1, sum sq, Linf, dangling sum
  double *hpart;       // hub segment partial sums
  uint32_t *hcnt;      // hub segment counters (indexed by the hub's first slot)
  double *trace;       // [max_iter][3] or null
};

// ---------------------------------------------------------------- host helpers
void set_error(const char *fmt, ...);
std::string &last_error_ref();

#define PR_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::prpull::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),       \
                          __FILE__, __LINE__);                                         \
      return PR_EDEVICE;                                                               \
    }                                                                                  \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Launchers (defined in the .hip files).
hipError_t launch_prepare(hipStream_t s, const int32_t *off, int64_t N, int4 *desc, unsigned long long *bsum,
                          unsigned long long *host_total);
int64_t scan_block_count(int64_t N);
hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, int64_t n, uint32_t v);

}  // namespace prpull
