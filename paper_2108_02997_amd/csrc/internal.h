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
// and whose row ids fall in one window of kRows rows; rows longer than kTile ("long rows") get
// tiles of their own, one per segment of at most kSeg entries.  A tile of short rows therefore
// spans fewer than 2*kTile entries.
constexpr int kTile = 1024;
constexpr int kRows = 512;
constexpr int kSpan = 2 * kTile;
constexpr int kRowsPerLane = kRows / kBlock;  // 2
constexpr int kSeg = 8192;
// Two partitions are kept per graph: A for the single-vector update (windows of kTile entries,
// kRows rows) and B for the K-column update, whose tiles stage whole gathered rows through LDS
// (windows of kTileB entries, kRowsB rows, so a tile spans fewer than kSpanB entries).
constexpr int kTileB = 256;
constexpr int kRowsB = 128;
constexpr int kSpanB = 2 * kTileB;
constexpr int kPartTile[2] = {kTile, kTileB};
constexpr int kPartRows[2] = {kRows, kRowsB};
// Smaller windows the autotuner may choose (the update kernels stage at most kSpan / kSpanB entries
// and kRows / kRowsB rows per tile, so any smaller window runs unchanged): partition A 1024/512,
// 512/256 or 256/128 entries/rows, partition B 256/128 or 128/64.  Prep buffers are sized for the
// smallest.
constexpr int kTuneBatchCols = 8;  // columns of the batch update the autotuner times
constexpr int kMinPartTile[2] = {256, 128};
constexpr int kMinPartRows[2] = {128, 64};
bool valid_window(int part, int tile, int rows);
// Default threshold: rows with in-degree above kMidDeg (and at most the tile window) are summed by
// a whole wave; pr_pull takes the threshold at run time (option "mid_deg", or the autotuner).
constexpr int kMidDeg = 32;
// The same for the pairs of the per-segment step (option "pair_mid_deg"): pairs are short (six
// entries on average on R-MAT scale 24 at 2^19-id segments) and a lane sums up to 256 of them
// faster than a wave pass does (1.73 against 1.77 ms per float64 update; 1024, never a wave:
// 1.97 ms).
constexpr int kPairMidDeg = 256;
// Upper bound of the update grid (blocks loop over tiles in a fixed round-robin order).
constexpr int kMaxGrid = 16384;
// Graphs of one many-graph batch.
constexpr int kMaxGraphs = 4096;
// The finishing kernel runs as one block of kFinBlock lanes.
constexpr int kFinBlock = 1024;
// Mixed precision, L1 norm: the float32 phase also hands over to float64 once the L1 change is
// below 2^-17, i.e. 128 float32 ulps of sum(r) = 1.  Closer to its rounding floor the float32
// iterate settles into a bias along the directions the update contracts only by alpha, and the
// float64 phase then needs many extra updates to remove it (R-MAT scale 22, alpha 0.85,
// tau 1e-10: 46 float32 + 27 float64 updates when waiting for tau, against 29 in float64 alone;
// handing over near 1e-5 needs no more updates than float64 alone).
constexpr double kL1Handover = 0x1p-17;

// ---------------------------------------------------------------- prep layout
// Tile descriptor: x = first row, y = first CSR entry, z = segment index (long row) or -1 (tile
// of short rows), w = partial slot of this segment for a hub, -1 otherwise.  Tile i ends where
// tile i+1 starts (rows desc[i].x .. desc[i+1].x, entries desc[i].y .. desc[i+1].y); a sentinel
// {N, E, -1, -1} follows the last tile.  Long rows of two or more segments ("hubs") are also
// listed in a hub table: x = row, y = segments, z = first slot.
struct PrepPart {
  int64_t desc_off;  // byte offset of the descriptors inside the prep buffer
  int64_t hub_off;   // byte offset of the hub table
  int32_t tile, rows, ndesc, nslots, nhubs, pad;
};

// Source-segmented layout (pr_prepare_segmented), in the same buffer after the plain prep's
// regions.  Source ids are cut into segments of seg_len consecutive ids; a pair is a run of one
// row's entries whose sources lie in one segment (at most kPairMax entries: longer runs are cut
// at row-relative multiples of kPairMax).  Pairs are listed segment by segment, rows ascending
// within a segment (the pair CSR: poff[P+1] over the permuted indices sidx[E]); the merge CSR
// lists, for every row, its pairs in segment order (moff[N+1] over mpos[P]).  part holds one
// partial sum per pair (float64, or float32 in a float32 phase) during a solve.
struct SegLayout {
  int64_t pairs;     // P
  int64_t poff_off;  // byte offsets of the arrays in the prep buffer
  int64_t moff_off;
  int64_t mpos_off;
  int64_t sidx_off;
  int64_t part_off;
  int64_t scan_off;  // scan scratch of the two tile partitions
  int64_t temp_off;  // construction scratch
  int64_t cub_off;   // hipCUB's storage inside it
  int64_t total;     // bytes of the whole buffer
  PrepPart pair_part;   // tiles over the pair CSR (no long rows)
  PrepPart merge_part;  // tiles over the merge CSR
  int64_t tsort_off;    // construction scratch of the tiles' sort (tile offsets, positions, hipCUB)
  int64_t tsort_bytes;
};
// Within a tile of the pair partition whose sources span fewer than 2^kRelBits ids, the entries
// are sorted by source and each sidx word packs (source - base) << kPosBits | position, position
// being the entry's place in the tile's pair order and base (the tile's smallest source) sitting
// in the tile descriptor's w; other tiles keep plain sources in pair order and w = -1.  The
// per-segment step then gathers in source order (neighbouring lanes share cache lines) and stages
// each value at its pair-order position, so every pair is still summed in its own order.
constexpr int32_t kPairMax = kTile;
// Tile window of the pair partition (entries).  Pairs are never long rows (kPairMax <= kPairTile),
// and a tile ends with a pair that starts inside its window, so it holds fewer than
// kPairTile + kPairMax entries: at most kSpan, the per-segment step's staging.
constexpr int kPairTile = kTile;
static_assert(kPairMax <= kPairTile && kPairTile + kPairMax <= kSpan, "pair tiles fit the staging");
constexpr int kPosBits = 11;
constexpr int kRelBits = 32 - kPosBits;
constexpr int32_t kMinSegLen = 256;

struct PrepHeader {
  int32_t magic;
  int32_t version;
  int64_t N;
  int64_t E;
  int32_t seg, pad;
  int64_t scan_off;   // byte offset of the scan scratch
  PrepPart part[2];
  int32_t seg_len;    // 0: no source-segmented layout, else source ids per segment
  int32_t pad2;
  SegLayout sl;
};
constexpr int32_t kPrepMagic = 0x50525032;  // "PRP2"
constexpr int32_t kPrepVersion = 4;

size_t prep_bytes(int64_t N, int64_t E);
int64_t max_desc(int64_t N, int64_t E, int tile, int rows);
int64_t max_slots(int64_t N, int64_t E);
int64_t max_hubs(int64_t N, int64_t E);

// ---------------------------------------------------------------- solve state (device)
// The first 16 bytes of every device solve state: what the host loop reads after a chunk.
struct LoopHead {
  int32_t stop;        // 1: the kernels of the running phase are no-ops
  int32_t phase_iter;  // updates performed in the running phase
  int32_t iter;        // updates performed so far (all phases)
  int32_t done;        // 1: the whole solve is finished
};

struct alignas(64) SolveState {
  LoopHead head;
  int32_t converged;  // 1: an update met tau in the convergence norm
  int32_t met32;      // the float32 phase met tau
  int32_t pad0, pad1;
  double c0;          // teleport term for the next update
  double err[3];      // L1, L2, Linf of the last update
  double prev_l1;     // L1 of the update before (float32 stagnation test)
};

// Damping-factor sweep as one power series (pr_pull_sweep).  From the uniform start u, the
// iterate of damping factor a after k updates is r_a(k) = a^k v_k + (1-a) sum_{j<k} a^j v_j, with
// v_j the iterates of the a = 1 update from u, and its change at update k is a^k (v_k - v_{k-1}):
// one a = 1 iteration serves every column.  Per-column parameters and stop state (device).
constexpr int kMaxSweepCols = 64;
constexpr int kSweepChunk = 32;  // updates between folds; the workspace keeps kSweepChunk + 1 iterates
struct SweepCols {
  double alpha[kMaxSweepCols];
  double tau[kMaxSweepCols];
  double err[kMaxSweepCols][3];     // the column's change at its last update
  double *ranks[kMaxSweepCols];     // output, accumulated fold by fold
  double *trace[kMaxSweepCols];     // [max_iter][3] or null
  int32_t norm[kMaxSweepCols];
  int32_t max_iter[kMaxSweepCols];
  int32_t stop_iter[kMaxSweepCols];  // 0 while the column runs, else the update it stopped at
  int32_t converged[kMaxSweepCols];
  int32_t K;
  int32_t remaining;
};

// Rank snapshots of a single-vector solve (the outputs row of section 3's tolerance study): the
// ranks at the first update whose change meets tau[i] in norm[i] -- the iterate a solve with that
// (tau, norm) would return -- are copied to out[i * N ..] as the solve runs, so one solve serves
// every (tau, norm) pair.  finalize marks the snapshots an update takes (pending, that update's
// output and its position in the chunk); k_snap, launched after it, copies them.
constexpr int kMaxSnaps = 64;
struct SnapTable {
  double tau[kMaxSnaps];
  int32_t norm[kMaxSnaps];
  int32_t iter[kMaxSnaps];     // the update snapshot i was taken at (0: not met yet)
  unsigned long long pending;  // snapshots taken at the last finalized update (bit i)
  const void *src;             // that update's output (y form, the solve's value type)
  double *out;                 // S x N ranks
  int32_t S;
  int32_t node;                // that update's position in its chunk
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
  int32_t mid_deg;     // rows of a tile with more entries are summed by a whole wave (<= kTile)
  SolveState *st;
  double *bpart;       // [grid][4] block partials: L1, sum sq, Linf, dangling sum
  double *hpart;       // hub segment partial sums
  const int4 *hubs;    // hub table
  int32_t nhubs;
  int32_t grid;        // number of blocks of the update launch (partials to reduce)
  double *trace;       // [max_iter][3] or null
  // Source-segmented update (poff null: the plain update).  Its per-segment step sums, over the
  // tiles pdesc, the entries sidx[poff[p] .. poff[p+1]) of pair p into partial[p] (type of the
  // phase); off / idx / desc / hubs then describe the merge step, in which row v sums
  // partial[idx[j]] over its entries j of off (its pairs in segment order).
  const int32_t *poff;
  const int32_t *sidx;
  const int4 *pdesc;
  void *partial;
  int32_t npdesc;
  int32_t pgrid;       // workgroups of the per-segment step
  int32_t seg_xcd;     // 1: the per-segment step gives each XCD a contiguous range of tiles
  int32_t merge_xcd;   // 1: the merge step does
  int32_t pair_mid_deg;  // pairs with more entries are summed by a whole wave (per-segment step)
  // Non-null: this is the a = 1 iteration of a power-series sweep; finalize decides every
  // column's stop instead of testing tau.
  SweepCols *sweep;
  // Non-null: rank snapshots are taken (finalize, k_snap); node is this update's position in its
  // chunk.
  SnapTable *snap;
  int32_t node;
  int32_t pad;
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
// host_total receives {descriptors, hub slots << 32 | hubs}.
hipError_t launch_prepare(hipStream_t s, int tile, int rows, const int32_t *off, int64_t N, int4 *desc, int4 *hubs,
                          void *scan, unsigned long long *host_total);
int64_t scan_block_count(int64_t N);
hipError_t launch_fill_u32(hipStream_t s, uint32_t *p, int64_t n, uint32_t v);
// The power-series sweep's fold and copy launchers: sweep.h.
// Source-segmented layout (segment.hip).
int64_t seg_count_blocks();
hipError_t launch_seg_count(hipStream_t s, const int32_t *off, const int32_t *idx, int32_t N, int32_t E,
                            int32_t seg_len, unsigned long long *block_counts, unsigned long long *host_total);
hipError_t seg_sort_temp_bytes(int64_t P, int key_bits, size_t *bytes);
hipError_t seg_scan_temp_bytes(int64_t n, size_t *bytes);
// Sort the entries of every pair tile by source and pack them with their pair-order positions.
hipError_t seg_tile_sort_temp_bytes(int64_t E, int64_t tiles, int key_bits, size_t *bytes);
size_t seg_tile_sort_scratch(int64_t E, int64_t tiles, size_t sort_bytes);
hipError_t launch_seg_tile_sort(hipStream_t s, int4 *pdesc, int32_t ndesc, int32_t E, int key_bits, char *base,
                                const SegLayout &sl);
hipError_t launch_seg_build(hipStream_t s, const int32_t *off, const int32_t *idx, int32_t N, int32_t E,
                            int32_t seg_len, int key_bits, int64_t P, char *base, const SegLayout &sl);

}  // namespace prpull
