// api_internal.h -- shared by the C-ABI translation units of libprpull.so (api*.hip): the
// context, workspace layouts, the graph-prep cache and the chunked iteration loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/prpull.h"
#include "batch.h"
#include "internal.h"
#include "multi.h"
#include "relabel.h"

namespace prpull {

std::string &last_error_ref();

// Kernel launchers and sizes (pull.hip, validate.hip, warmstart.hip).
hipError_t launch_init(hipStream_t s, bool fp32, const int32_t *outdeg, int32_t N, const double *init, void *y,
                       double alpha, SolveState *st, double *bpart, int64_t bpart_cap);
hipError_t launch_update(hipStream_t s, bool fp32, unsigned grid, const IterParams &p);
int update_blocks_per_cu(bool fp32);
hipError_t launch_convert(hipStream_t s, const float *y32, double *y64, int32_t N, SolveState *st);
hipError_t launch_l1(hipStream_t s, const double *x, const double *y, int64_t N, double *part, int32_t nb);
int mlp_param_count();
int mlp_backward_blocks(int64_t N);
hipError_t launch_features(hipStream_t s, const int32_t *off, const int32_t *idx, const int32_t *outdeg, int32_t N,
                           const int4 *desc, int32_t ndesc, const int4 *hubs, int32_t nhubs, const double *r,
                           double alpha_t, float *feat, const double *r_target, float *target);
hipError_t launch_mlp_forward(hipStream_t s, const float *W, const float *feat, int64_t N, float *y, uint16_t *act);
hipError_t launch_mlp_backward(hipStream_t s, const float *W, const float *feat, const uint16_t *act, const float *y,
                               const float *target, int64_t N, float *part, double *loss_part, float *dW,
                               double *loss);
hipError_t launch_adam(hipStream_t s, float *W, const float *g, float *m, float *v, int32_t n, float lr, float beta1,
                       float beta2, float eps, int32_t step);
hipError_t launch_start_vector(hipStream_t s, const float *feat, const float *y, int64_t N, double *r0, double *part);
hipError_t launch_output(hipStream_t s, bool fp32, const int32_t *outdeg, const void *y, int32_t N, double *ranks);
hipError_t launch_snap(hipStream_t s, bool fp32, const IterParams &p);
hipError_t launch_validate(hipStream_t s, const int32_t *off, const int32_t *idx, const int32_t *outdeg, int32_t N,
                           int32_t E, uint32_t *cnt, int32_t *flags, int32_t *host_flags);

struct GraphEntry {
  std::vector<unsigned char> key;
  hipGraphExec_t exec;
  uint64_t last_use;
  std::vector<hipEvent_t> events;  // unused (kept empty)
};

// One chunk of a solve loop: `count` launches of one update kernel; launch(s, k) issues the
// k-th.  `key` identifies the captured graph (kernel, parameters, buffers).
struct ChunkSpec {
  int kind;
  int sub_kind = -1;  // also counted under this kind (the batch kernels by columns per lane)
  int count;
  std::vector<unsigned char> key;
  std::function<hipError_t(hipStream_t, int)> launch;
};

}  // namespace prpull

using namespace prpull;

// The autotuner's choice for a graph's source-segmented update.
struct SegTune {
  int32_t pair_mid_deg, seg_grid, merge_xcd;
};

struct pr_ctx {
  int device = 0;
  hipStream_t capture = nullptr;  // private stream used only for graph capture
  SolveState *hstate = nullptr;   // pinned host copy of the solve state
  unsigned long long *hscratch = nullptr;  // pinned host words for small read-backs
  BatchCols *hcols = nullptr;             // pinned staging of per-column parameters
  SweepCols *hsweep = nullptr;            // pinned staging of a sweep's column table
  BatchState *hbstate = nullptr;          // pinned host copy of a batch state
  void *hmulti = nullptr;                 // pinned staging of many-graph tables
  size_t hmulti_bytes = 0;
  std::map<const void *, PrepHeader> preps;  // prep buffers prepared in this context
  std::vector<GraphEntry> graphs;
  uint64_t clock = 0;
  // tunables (pr_set_option)
  int64_t max_grid = 0;     // 0: one workgroup per resident slot (compute units x occupancy)
  int64_t resident[2] = {1, 1};  // resident update workgroups: [float64, float32]
  int64_t seg_grid = 0;     // workgroups of the per-segment step; 0: the update's resident count
  int64_t pair_mid_deg = kPairMidDeg;  // wave-per-pair threshold of the per-segment step
  bool pair_mid_deg_set = false, seg_grid_set = false, merge_xcd_set = false;  // set explicitly
  // (graph signature, segment length) -> the autotuner's segmented-update settings
  std::map<std::vector<int64_t>, SegTune> tuned_seg;
  int64_t chunk = 16;
  int64_t loop_mode = 0;  // 0: HIP-graph chunks, 1: direct launches
  int64_t timing = 0;     // 1: bracket every update launch with HIP events
  int64_t batch_chunk = 2;  // updates between host checks of a batch solve (compaction points)
  int64_t mid_deg = kMidDeg;  // lane-per-row / wave-per-row threshold of pr_pull
  bool mid_deg_set = false;   // set explicitly (overrides the autotuner's choice)
  int64_t use_tuned = 1;      // 1: use autotuned settings of graphs with a known signature
  std::map<std::vector<int64_t>, std::pair<int32_t, int32_t>> tuned;  // signature -> (mid_deg, grid)
  // signature -> (wave-per-row threshold, workgroups per resident slot) of pr_pull_batch
  std::map<std::vector<int64_t>, std::pair<int32_t, int32_t>> tuned_batch;
  std::string tune_file;
  int64_t compact = 1;      // 1: repack the active columns of a batch into narrower rows
  int64_t narrow = 1;       // 1: one or two columns run on rows of one or two values
  int64_t handover32 = 1;   // 1: the first float64 update of a mixed batch reads float32 rows
  int64_t segmented = 1;    // 1: pr_pull uses the source-segmented layout of a prep that has one
  int64_t seg_xcd = 1;      // 1: the per-segment step gives each XCD a contiguous range of tiles
  int64_t merge_xcd = 0;    // 1: the merge step does too
  int64_t window_tile[2] = {kTile, kTileB};  // tile windows of new partitions A and B (entries)
  int64_t window_rows[2] = {kRows, kRowsB};
  int64_t barrier_ms = 5000;  // time limit of a grid-barrier wait in pr_pull_multi
  std::vector<hipEvent_t> direct_events;
  int64_t stat_launches[PR_KERNEL_KINDS] = {};
  double stat_ms[PR_KERNEL_KINDS] = {};
};

namespace prpull {

// Two HIP events owned by a scope.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() = default;
  EventPair(const EventPair &) = delete;
  EventPair &operator=(const EventPair &) = delete;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

struct Carver {
  char *base;
  size_t used = 0;
  explicit Carver(void *b) : base((char *)b) {}
  void *take(size_t n) {
    void *p = base ? base + used : nullptr;
    used += align_up(n, 256);
    return p;
  }
};

// Workspace layout of one solve.
struct Layout {
  SolveState *st;
  double *bpart;
  double *hpart;
  SnapTable *snap;
  double *y64[2];
  float *y32[2];
  void *prep;
  size_t total;
};

// Workspace layout of a K-column solve.
struct BatchLayout {
  BatchState *st;
  BatchCols *cols;
  double *bpart;
  double *hpart;
  double *hacc;
  float *y32[2];
  double *y64[2];
  void *prep;
  size_t total;
};

// Workspace carving, graph prep and the chunked iteration loop (api.hip).
bool bad_graph_sizes(int64_t N, int64_t E);
Layout carve(void *ws, int64_t N, int64_t E, int32_t precision, bool with_prep);
int prepare_into(pr_ctx *ctx, hipStream_t s, const int32_t *off, int64_t N, int64_t E, void *prep, PrepHeader *out);
int get_prep(pr_ctx *ctx, hipStream_t s, const void *prep, int64_t N, int64_t E, PrepHeader *out);
int prepare_parts(pr_ctx *ctx, hipStream_t s, const int32_t *off, int64_t N, int64_t E, void *prep, int tile_a,
                  int tile_b, PrepHeader *hin, PrepHeader *out);
int write_prep_header(pr_ctx *ctx, hipStream_t s, void *prep, const PrepHeader &h);
int seg_key_bits(int64_t N, int32_t seg_len);
bool seg_layout(int64_t N, int64_t E, int32_t seg_len, int64_t P, SegLayout *sl);
int make_events(std::vector<hipEvent_t> &ev, size_t n);
int run_chunk(pr_ctx *ctx, hipStream_t s, const ChunkSpec &c, const std::vector<hipEvent_t> **events);
int run_until_stop(pr_ctx *ctx, hipStream_t s, const ChunkSpec &c, const LoopHead *head, int max_updates,
                   int *final_buf);
ChunkSpec update_chunk(pr_ctx *ctx, bool fp32, unsigned grid, const IterParams &p, void *b0, void *b1);
int batch_row_width(int K, bool fp32, bool narrow);
BatchLayout carve_batch(void *ws, int64_t N, int64_t E, int32_t K, int32_t precision, bool with_prep);
ChunkSpec batch_chunk(pr_ctx *ctx, bool fp32, int kp, unsigned grid, const BatchParams &p, void *b0, void *b1);
std::vector<int64_t> graph_signature(const PrepHeader &h);
std::pair<int32_t, int64_t> tuned_settings(pr_ctx *ctx, const PrepHeader &h);
std::vector<int64_t> seg_signature(const PrepHeader &h);
std::pair<int32_t, int32_t> tuned_batch_settings(pr_ctx *ctx, const PrepHeader &h);
void load_tune_file(pr_ctx *ctx);
void save_tune_entry(pr_ctx *ctx, const std::vector<int64_t> &sig, int32_t mid, int32_t grid, int32_t mid_b,
                     int32_t grid_b);
void save_tune_seg_entry(pr_ctx *ctx, const std::vector<int64_t> &sig, const SegTune &t);
// The rank snapshots a pr_pull_snapshots call asks for (tau, norm and iter: host; out: device).
struct SnapRequest {
  int32_t S;
  const double *tau;
  const int32_t *norm;
  double *out;
  int32_t *iter;
};
int pull_solve(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
               int64_t N, int64_t E, const void *prep, double alpha, double tau, int32_t norm, int32_t max_iter,
               int32_t precision, const double *init, double *ranks, double *norm_trace, void *workspace,
               size_t workspace_bytes, pr_result *out, const SnapRequest *snaps = nullptr);
// The library's fixed device scratch (api_noalloc.hip): its address on `device`, resolved once
// per device; PR_OK or PR_EDEVICE.
int scratch_setup(int device);

}  // namespace prpull
