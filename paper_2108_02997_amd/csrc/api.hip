// api.hip -- the C ABI of libprpull.so (declared in include/prpull.h): argument checks,
// workspace carving, graph prep caching and the on-device-convergence iteration loop.
//
// The loop: updates are launched in chunks of `chunk` kernels, alternating the two iterate
// buffers.  A chunk is captured once into a HIP graph (on a private capture stream) and
// replayed on the caller's stream; once an update meets the stopping rule the remaining
// kernels of the chunk return at entry.  After each chunk the host reads the 64-byte solve
// state from pinned memory and stops when the device says so.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/prpull.h"
#include "batch.h"
#include "internal.h"
#include "multi.h"
#include "relabel.h"

namespace prpull {

std::string &last_error_ref() {
  static thread_local std::string s;
  return s;
}

void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error_ref() = buf;
}

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

struct pr_ctx {
  int device = 0;
  hipStream_t capture = nullptr;  // private stream used only for graph capture
  SolveState *hstate = nullptr;   // pinned host copy of the solve state
  unsigned long long *hscratch = nullptr;  // pinned host words for small read-backs
  BatchCols *hcols = nullptr;             // pinned staging of per-column parameters
  BatchState *hbstate = nullptr;          // pinned host copy of a batch state
  void *hmulti = nullptr;                 // pinned staging of many-graph tables
  size_t hmulti_bytes = 0;
  std::map<const void *, PrepHeader> preps;  // prep buffers prepared in this context
  std::vector<GraphEntry> graphs;
  uint64_t clock = 0;
  // tunables (pr_set_option)
  int64_t max_grid = 0;     // 0: one workgroup per resident slot (compute units x occupancy)
  int64_t resident[2] = {1, 1};  // resident update workgroups: [float64, float32]
  int64_t chunk = 8;
  int64_t loop_mode = 0;  // 0: HIP-graph chunks, 1: direct launches
  int64_t timing = 0;     // 1: bracket every update launch with HIP events
  int64_t batch_chunk = 2;  // updates between host checks of a batch solve (compaction points)
  int64_t mid_deg = kMidDeg;  // lane-per-row / wave-per-row threshold of pr_pull
  bool mid_deg_set = false;   // set explicitly (overrides the autotuner's choice)
  int64_t use_tuned = 1;      // 1: use autotuned settings of graphs with a known signature
  std::map<std::vector<int64_t>, std::pair<int32_t, int32_t>> tuned;  // signature -> (mid_deg, grid)
  std::string tune_file;
  int64_t compact = 1;      // 1: repack the active columns of a batch into narrower rows
  int64_t narrow = 1;       // 1: one or two columns run on rows of one or two values
  int64_t barrier_ms = 5000;  // time limit of a grid-barrier wait in pr_pull_multi
  std::vector<hipEvent_t> direct_events;
  int64_t stat_launches[PR_KERNEL_KINDS] = {};
  double stat_ms[PR_KERNEL_KINDS] = {};
};

namespace {

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

bool bad_graph_sizes(int64_t N, int64_t E) {
  if (N < 1 || N > 2147483646LL) {
    set_error("N must be in [1, 2^31-2], got %lld", (long long)N);
    return true;
  }
  if (E < 0 || E > 2147483647LL) {
    set_error("E must be in [0, 2^31-1], got %lld", (long long)E);
    return true;
  }
  return false;
}

// Workspace layout of one solve.
struct Layout {
  SolveState *st;
  double *bpart;
  double *hpart;
  double *y64[2];
  float *y32[2];
  void *prep;
  size_t total;
};

Layout carve(void *ws, int64_t N, int64_t E, int32_t precision, bool with_prep) {
  Carver c(ws);
  Layout L{};
  L.st = (SolveState *)c.take(sizeof(SolveState));
  L.bpart = (double *)c.take(4 * sizeof(double) * (size_t)kMaxGrid);
  const int64_t slots = max_slots(N, E);
  L.hpart = (double *)c.take(sizeof(double) * (size_t)slots);
  L.y64[0] = (double *)c.take(sizeof(double) * (size_t)N);
  L.y64[1] = (double *)c.take(sizeof(double) * (size_t)N);
  if (precision == PR_MIXED || precision == PR_FP32) {
    L.y32[0] = (float *)c.take(sizeof(float) * (size_t)N);
    L.y32[1] = (float *)c.take(sizeof(float) * (size_t)N);
  }
  L.prep = with_prep ? c.take(prep_bytes(N, E)) : nullptr;
  L.total = c.used;
  return L;
}

int prepare_into(pr_ctx *ctx, hipStream_t s, const int32_t *off, int64_t N, int64_t E, void *prep,
                 PrepHeader *out) {
  PrepHeader h{};
  h.magic = kPrepMagic;
  h.version = 2;
  h.N = N;
  h.E = E;
  h.seg = kSeg;
  int64_t o = (int64_t)align_up(sizeof(PrepHeader), 256);
  for (int i = 0; i < 2; ++i) {
    PrepPart &pp = h.part[i];
    pp.tile = kPartTile[i];
    pp.rows = kPartRows[i];
    pp.desc_off = o;
    o += (int64_t)align_up((size_t)(max_desc(N, E, pp.tile, pp.rows) + 1) * sizeof(int4), 256);
    pp.hub_off = o;
    o += (int64_t)align_up((size_t)max_hubs(N, E) * sizeof(int4), 256);
  }
  h.scan_off = o;
  char *base = (char *)prep;
  for (int i = 0; i < 2; ++i) {
    PrepPart &pp = h.part[i];
    PR_HIP(launch_prepare(s, i, off, N, (int4 *)(base + pp.desc_off), (int4 *)(base + pp.hub_off), base + h.scan_off,
                          ctx->hscratch));
    const unsigned long long tot_a = ctx->hscratch[0], tot_b = ctx->hscratch[1];
    pp.ndesc = (int32_t)tot_a;
    pp.nslots = (int32_t)(tot_b >> 32);
    pp.nhubs = (int32_t)(tot_b & 0xffffffffull);
    if (pp.ndesc < 1 || pp.ndesc > max_desc(N, E, pp.tile, pp.rows) || pp.nslots > max_slots(N, E) ||
        pp.nhubs > max_hubs(N, E)) {
      set_error("internal: tile partition %d out of bounds (ndesc %d, slots %d, hubs %d)", i, pp.ndesc, pp.nslots,
                pp.nhubs);
      return PR_EDEVICE;
    }
  }
  memcpy(ctx->hscratch + 8, &h, sizeof h);
  PR_HIP(hipMemcpyAsync(prep, ctx->hscratch + 8, sizeof h, hipMemcpyHostToDevice, s));
  PR_HIP(hipStreamSynchronize(s));
  ctx->preps[prep] = h;
  *out = h;
  return PR_OK;
}

int get_prep(pr_ctx *ctx, hipStream_t s, const void *prep, int64_t N, int64_t E, PrepHeader *out) {
  auto it = ctx->preps.find(prep);
  PrepHeader h{};
  if (it != ctx->preps.end()) {
    h = it->second;
  } else {
    PR_HIP(hipMemcpyAsync(ctx->hscratch + 8, prep, sizeof h, hipMemcpyDeviceToHost, s));
    PR_HIP(hipStreamSynchronize(s));
    memcpy(&h, ctx->hscratch + 8, sizeof h);
  }
  if (h.magic != kPrepMagic || h.version != 2) {
    set_error("prep buffer was not written by pr_prepare");
    return PR_EINVAL;
  }
  if (h.N != N || h.E != E || h.seg != kSeg || h.part[0].tile != kTile || h.part[1].tile != kTileB) {
    set_error("prep buffer belongs to another graph (N=%lld E=%lld, expected N=%lld E=%lld)", (long long)h.N,
              (long long)h.E, (long long)N, (long long)E);
    return PR_EINVAL;
  }
  *out = h;
  return PR_OK;
}

int make_events(std::vector<hipEvent_t> &ev, size_t n) {
  while (ev.size() < n) {
    hipEvent_t e;
    PR_HIP(hipEventCreate(&e));
    ev.push_back(e);
  }
  return PR_OK;
}

// Issue one chunk on stream s (captured graph or direct launches); *events receives the
// timestamps bracketing each launch when timing is on, else nullptr.
int run_chunk(pr_ctx *ctx, hipStream_t s, const ChunkSpec &c, const std::vector<hipEvent_t> **events) {
  *events = nullptr;
  const bool timed = ctx->timing != 0;
  // events recorded inside a captured graph cannot be timed, so timed chunks launch one by one
  if (ctx->loop_mode == 1 || timed) {
    if (timed) {
      int rc = make_events(ctx->direct_events, (size_t)c.count + 1);
      if (rc != PR_OK) return rc;
      PR_HIP(hipEventRecord(ctx->direct_events[0], s));
    }
    for (int k = 0; k < c.count; ++k) {
      PR_HIP(c.launch(s, k));
      if (timed) PR_HIP(hipEventRecord(ctx->direct_events[k + 1], s));
    }
    if (timed) *events = &ctx->direct_events;
    return PR_OK;
  }
  std::vector<unsigned char> key = c.key;
  const int64_t meta[2] = {c.kind, c.count};
  key.insert(key.end(), (const unsigned char *)meta, (const unsigned char *)meta + sizeof meta);
  GraphEntry *entry = nullptr;
  for (auto &g : ctx->graphs)
    if (g.key == key) {
      g.last_use = ++ctx->clock;
      entry = &g;
    }
  if (!entry) {
    std::vector<hipEvent_t> ev;
    hipGraph_t g = nullptr;
    PR_HIP(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int k = 0; k < c.count && err == hipSuccess; ++k) err = c.launch(ctx->capture, k);
    hipError_t e2 = hipStreamEndCapture(ctx->capture, &g);
    hipGraphExec_t exec = nullptr;
    if (err == hipSuccess && e2 == hipSuccess) err = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (err != hipSuccess || e2 != hipSuccess) {
      for (auto e : ev) (void)hipEventDestroy(e);
      set_error("graph capture failed: %s", hipGetErrorString(err != hipSuccess ? err : e2));
      return PR_EDEVICE;
    }
    constexpr size_t kMaxCachedGraphs = 48;  // instantiated update chunks kept per context
    if (ctx->graphs.size() >= kMaxCachedGraphs) {
      size_t lru = 0;
      for (size_t i = 1; i < ctx->graphs.size(); ++i)
        if (ctx->graphs[i].last_use < ctx->graphs[lru].last_use) lru = i;
      (void)hipGraphExecDestroy(ctx->graphs[lru].exec);
      for (auto e : ctx->graphs[lru].events) (void)hipEventDestroy(e);
      ctx->graphs.erase(ctx->graphs.begin() + (long)lru);
    }
    ctx->graphs.push_back(GraphEntry{key, exec, ++ctx->clock, ev});
    entry = &ctx->graphs.back();
  }
  PR_HIP(hipGraphLaunch(entry->exec, s));
  return PR_OK;
}

// Replay chunks until the device sets head.stop; `head` is the device LoopHead of the solve.
// Returns the parity of the updates done in the phase (index of the buffer holding the newest
// iterate when updates alternate two buffers starting from buffer 0).
int run_until_stop(pr_ctx *ctx, hipStream_t s, const ChunkSpec &c, const LoopHead *head, int max_updates,
                   int *final_buf) {
  LoopHead *h = (LoopHead *)ctx->hstate;
  int before = 0;
  for (int rounds = 0;; ++rounds) {
    const std::vector<hipEvent_t> *ev = nullptr;
    int rc = run_chunk(ctx, s, c, &ev);
    if (rc != PR_OK) return rc;
    PR_HIP(hipMemcpyAsync(h, head, sizeof(LoopHead), hipMemcpyDeviceToHost, s));
    PR_HIP(hipStreamSynchronize(s));
    const int did = h->phase_iter - before;
    if (ev && did > 0) {
      float ms = 0.f;
      for (int k = 0; k < did && k < c.count; ++k) {
        PR_HIP(hipEventElapsedTime(&ms, (*ev)[k], (*ev)[k + 1]));
        ctx->stat_ms[c.kind] += ms;
        ctx->stat_launches[c.kind] += 1;
        if (c.sub_kind >= 0) {
          ctx->stat_ms[c.sub_kind] += ms;
          ctx->stat_launches[c.sub_kind] += 1;
        }
      }
    }
    before = h->phase_iter;
    if (h->stop) break;
    if (rounds > max_updates) {  // cannot happen: the kernels stop at max_iter
      set_error("internal: update limit passed without stop");
      return PR_EDEVICE;
    }
  }
  *final_buf = h->phase_iter & 1;
  return PR_OK;
}

ChunkSpec update_chunk(pr_ctx *ctx, bool fp32, unsigned grid, const IterParams &p, void *b0, void *b1) {
  ChunkSpec c;
  c.kind = fp32 ? PR_KERNEL_UPDATE_F32 : PR_KERNEL_UPDATE_F64;
  c.count = (int)ctx->chunk;
  IterParams q = p;
  q.y_in = b0;
  q.y_out = b1;
  const int64_t g = grid;
  c.key.resize(sizeof q + sizeof g);
  memcpy(c.key.data(), &q, sizeof q);
  memcpy(c.key.data() + sizeof q, &g, sizeof g);
  c.launch = [fp32, grid, p, b0, b1](hipStream_t s, int k) {
    IterParams r = p;
    r.y_in = (k & 1) ? b1 : b0;
    r.y_out = (k & 1) ? b0 : b1;
    return launch_update(s, fp32, grid, r);
  };
  return c;
}

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

// Row width (values per vertex) of the batch state for K columns: 1 or 2 (narrow rows, one lane
// per row fetch), else 4, 8, 12 or 16.  For float32 a 64-byte row is preferred over a 48-byte one
// once K > 8: a row fetch then touches exactly one 64-byte line.
int batch_row_width(int K, bool fp32, bool narrow) {
  if (narrow && K <= 2) return K < 1 ? 1 : K;
  if (fp32 && K > 8) return 16;
  return 4 * ((K + 3) / 4);
}

// Index of a row width among the per-width stats kinds (widths 1, 2, 4, 8, 12, 16).
static int width_index(int kp) { return kp == 1 ? 0 : kp == 2 ? 1 : kp / 4 + 1; }

BatchLayout carve_batch(void *ws, int64_t N, int64_t E, int32_t K, int32_t precision, bool with_prep) {
  Carver c(ws);
  BatchLayout L{};
  // sized for the widest layout of K columns (narrow rows only ever take less)
  const int64_t kp32 = batch_row_width(K, true, false), kp64 = batch_row_width(K, false, false);
  L.st = (BatchState *)c.take(sizeof(BatchState));
  L.cols = (BatchCols *)c.take(sizeof(BatchCols));
  L.bpart = (double *)c.take(sizeof(double) * 4 * kMaxCols * (size_t)kMaxGrid);
  L.hpart = (double *)c.take(sizeof(double) * kMaxCols * (size_t)max_slots(N, E));
  L.hacc = (double *)c.take(sizeof(double) * 4 * kMaxCols * (size_t)hub_blocks(max_hubs(N, E)));
  if (precision == PR_MIXED) {
    L.y32[0] = (float *)c.take(sizeof(float) * (size_t)(N * kp32));
    L.y32[1] = (float *)c.take(sizeof(float) * (size_t)(N * kp32));
  }
  L.y64[0] = (double *)c.take(sizeof(double) * (size_t)(N * kp64));
  L.y64[1] = (double *)c.take(sizeof(double) * (size_t)(N * kp64));
  L.prep = with_prep ? c.take(prep_bytes(N, E)) : nullptr;
  L.total = c.used;
  return L;
}

ChunkSpec batch_chunk(pr_ctx *ctx, bool fp32, int kp, unsigned grid, const BatchParams &p, void *b0, void *b1) {
  ChunkSpec c;
  c.kind = fp32 ? PR_KERNEL_BATCH_F32 : PR_KERNEL_BATCH_F64;
  c.sub_kind = (fp32 ? PR_KERNEL_BATCH_F32_W1 : PR_KERNEL_BATCH_F64_W1) + width_index(kp);
  c.count = (int)ctx->chunk;
  BatchParams q = p;
  q.y_in = b0;
  q.y_out = b1;
  const int64_t meta[2] = {grid, kp};
  c.key.resize(sizeof q + sizeof meta);
  memcpy(c.key.data(), &q, sizeof q);
  memcpy(c.key.data() + sizeof q, meta, sizeof meta);
  c.launch = [fp32, kp, grid, p, b0, b1](hipStream_t s, int k) {
    BatchParams r = p;
    r.y_in = (k & 1) ? b1 : b0;
    r.y_out = (k & 1) ? b0 : b1;
    return launch_batch_update(s, fp32, kp, grid, r);
  };
  return c;
}

// Graph signature for the autotuner's table: sizes and the tile counts of both partitions.
std::vector<int64_t> graph_signature(const PrepHeader &h) {
  return {h.N, h.E, h.part[0].ndesc, h.part[0].nhubs, h.part[0].nslots, h.part[1].ndesc};
}

// (mid_deg, grid cap) for a graph: explicit options first, then the autotuner's table, then defaults.
std::pair<int32_t, int64_t> tuned_settings(pr_ctx *ctx, const PrepHeader &h) {
  int32_t mid = (int32_t)ctx->mid_deg;
  int64_t grid = ctx->max_grid;
  if (ctx->use_tuned) {
    auto it = ctx->tuned.find(graph_signature(h));
    if (it != ctx->tuned.end()) {
      if (!ctx->mid_deg_set) mid = it->second.first;
      if (ctx->max_grid == 0) grid = it->second.second;
    }
  }
  return {mid, grid};
}

void load_tune_file(pr_ctx *ctx) {
  const char *f = getenv("PRPULL_TUNE_FILE");
  if (!f || !*f) return;
  ctx->tune_file = f;
  FILE *fp = fopen(f, "r");
  if (!fp) return;
  long long s[6];
  int m, g;
  while (fscanf(fp, "%lld %lld %lld %lld %lld %lld %d %d", &s[0], &s[1], &s[2], &s[3], &s[4], &s[5], &m, &g) == 8)
    ctx->tuned[{s[0], s[1], s[2], s[3], s[4], s[5]}] = {m, g};
  fclose(fp);
}

void save_tune_entry(pr_ctx *ctx, const std::vector<int64_t> &sig, int32_t mid, int32_t grid) {
  if (ctx->tune_file.empty()) return;
  FILE *fp = fopen(ctx->tune_file.c_str(), "a");
  if (!fp) return;
  fprintf(fp, "%lld %lld %lld %lld %lld %lld %d %d\n", (long long)sig[0], (long long)sig[1], (long long)sig[2],
          (long long)sig[3], (long long)sig[4], (long long)sig[5], mid, grid);
  fclose(fp);
}

}  // namespace

extern "C" {

const char *pr_last_error(void) { return last_error_ref().c_str(); }

const char *pr_version(void) { return "prpull 0.1 (gfx950)"; }

int pr_create(pr_ctx **out, int device) {
  if (!out) {
    set_error("pr_create: out is NULL");
    return PR_EINVAL;
  }
  *out = nullptr;
  int n = 0;
  PR_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) {
    set_error("pr_create: device %d not present (%d devices)", device, n);
    return PR_EDEVICE;
  }
  DeviceGuard g(device);
  pr_ctx *c = new pr_ctx();
  c->device = device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  c->resident[0] = (int64_t)cus * update_blocks_per_cu(false);
  c->resident[1] = (int64_t)cus * update_blocks_per_cu(true);
  load_tune_file(c);
  hipError_t e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hstate, sizeof(SolveState), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hscratch, 64 * sizeof(unsigned long long), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hcols, sizeof(BatchCols), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hbstate, sizeof(BatchState), hipHostMallocDefault);
  if (e != hipSuccess) {
    set_error("pr_create: %s", hipGetErrorString(e));
    if (c->capture) (void)hipStreamDestroy(c->capture);
    if (c->hstate) (void)hipHostFree(c->hstate);
    if (c->hscratch) (void)hipHostFree(c->hscratch);
    if (c->hcols) (void)hipHostFree(c->hcols);
    if (c->hbstate) (void)hipHostFree(c->hbstate);
    delete c;
    return PR_EDEVICE;
  }
  *out = c;
  return PR_OK;
}

void pr_destroy(pr_ctx *ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  for (auto &e : ctx->graphs) {
    (void)hipGraphExecDestroy(e.exec);
    for (auto ev : e.events) (void)hipEventDestroy(ev);
  }
  for (auto ev : ctx->direct_events) (void)hipEventDestroy(ev);
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  if (ctx->hstate) (void)hipHostFree(ctx->hstate);
  if (ctx->hscratch) (void)hipHostFree(ctx->hscratch);
  if (ctx->hcols) (void)hipHostFree(ctx->hcols);
  if (ctx->hbstate) (void)hipHostFree(ctx->hbstate);
  if (ctx->hmulti) (void)hipHostFree(ctx->hmulti);
  delete ctx;
}

int pr_set_option(pr_ctx *ctx, const char *key, int64_t value) {
  if (!ctx || !key) {
    set_error("pr_set_option: NULL argument");
    return PR_EINVAL;
  }
  if (!strcmp(key, "grid")) {
    if (value < 0 || value > kMaxGrid) {
      set_error("grid must be in [0, %d] (0 = resident workgroups)", kMaxGrid);
      return PR_EINVAL;
    }
    ctx->max_grid = value;
  } else if (!strcmp(key, "chunk")) {
    if (value < 2 || value > 64 || (value & 1)) {
      set_error("chunk must be even and in [2, 64]");
      return PR_EINVAL;
    }
    ctx->chunk = value;
  } else if (!strcmp(key, "mid_deg")) {
    if (value < 0 || value > kTile) {
      set_error("mid_deg must be in [0, %d]", kTile);
      return PR_EINVAL;
    }
    ctx->mid_deg = value;
    ctx->mid_deg_set = true;
  } else if (!strcmp(key, "tuned")) {
    if (value != 0 && value != 1) {
      set_error("tuned must be 0 or 1");
      return PR_EINVAL;
    }
    ctx->use_tuned = value;
  } else if (!strcmp(key, "batch_chunk")) {
    if (value < 1 || value > 64) {
      set_error("batch_chunk must be in [1, 64]");
      return PR_EINVAL;
    }
    ctx->batch_chunk = value;
  } else if (!strcmp(key, "compact")) {
    if (value != 0 && value != 1) {
      set_error("compact must be 0 or 1");
      return PR_EINVAL;
    }
    ctx->compact = value;
  } else if (!strcmp(key, "narrow")) {
    if (value != 0 && value != 1) {
      set_error("narrow must be 0 or 1");
      return PR_EINVAL;
    }
    ctx->narrow = value;
  } else if (!strcmp(key, "barrier_ms")) {
    if (value < 0 || value > 600000) {
      set_error("barrier_ms must be in [0, 600000]");
      return PR_EINVAL;
    }
    ctx->barrier_ms = value;
  } else if (!strcmp(key, "timing")) {
    if (value != 0 && value != 1) {
      set_error("timing must be 0 or 1");
      return PR_EINVAL;
    }
    ctx->timing = value;
  } else if (!strcmp(key, "loop")) {
    if (value != 0 && value != 1) {
      set_error("loop must be 0 (graph) or 1 (direct)");
      return PR_EINVAL;
    }
    ctx->loop_mode = value;
  } else {
    set_error("unknown option '%s'", key);
    return PR_EINVAL;
  }
  return PR_OK;
}

int pr_get_stats(pr_ctx *ctx, int32_t kind, int64_t *launches, double *milliseconds) {
  if (!ctx || !launches || !milliseconds || kind < 0 || kind >= PR_KERNEL_KINDS) {
    set_error("pr_get_stats: bad argument");
    return PR_EINVAL;
  }
  *launches = ctx->stat_launches[kind];
  *milliseconds = ctx->stat_ms[kind];
  return PR_OK;
}

int pr_reset_stats(pr_ctx *ctx) {
  if (!ctx) {
    set_error("pr_reset_stats: NULL context");
    return PR_EINVAL;
  }
  for (int k = 0; k < PR_KERNEL_KINDS; ++k) {
    ctx->stat_launches[k] = 0;
    ctx->stat_ms[k] = 0.0;
  }
  return PR_OK;
}

size_t pr_prep_bytes(int64_t N, int64_t E) {
  if (bad_graph_sizes(N, E)) return 0;
  return prep_bytes(N, E);
}

int pr_prepare(pr_ctx *ctx, void *stream, const int32_t *in_offsets, int64_t N, int64_t E, void *prep,
               size_t prep_bytes_) {
  if (!ctx || !in_offsets || !prep) {
    set_error("pr_prepare: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  if (prep_bytes_ < prep_bytes(N, E)) {
    set_error("pr_prepare: prep buffer has %zu bytes, needs %zu", prep_bytes_, prep_bytes(N, E));
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  PrepHeader h;
  return prepare_into(ctx, (hipStream_t)stream, in_offsets, N, E, prep, &h);
}

int pr_validate_graph(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                      const int32_t *outdeg, int64_t N, int64_t E, void *workspace, size_t workspace_bytes) {
  if (!ctx || !in_offsets || !outdeg || !workspace || (E > 0 && !in_indices)) {
    set_error("pr_validate_graph: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  const size_t need = align_up(4 * (size_t)N, 256) + 256;
  if (workspace_bytes < need) {
    set_error("pr_validate_graph: workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  uint32_t *cnt = (uint32_t *)workspace;
  int32_t *flags = (int32_t *)((char *)workspace + align_up(4 * (size_t)N, 256));
  int32_t *hf = (int32_t *)ctx->hscratch;
  PR_HIP(launch_validate((hipStream_t)stream, in_offsets, in_indices, outdeg, (int32_t)N, (int32_t)E, cnt, flags, hf));
  if (hf[0] || hf[1] || hf[2]) {
    set_error("malformed CSR:%s%s%s (first offending offset %d, index position %d, vertex %d)",
              hf[0] ? " offsets" : "", hf[1] ? " indices" : "", hf[2] ? " out-degrees" : "", hf[0] ? hf[3] : -1,
              hf[1] ? hf[4] : -1, hf[2] ? hf[5] : -1);
    return PR_EGRAPH;
  }
  return PR_OK;
}

size_t pr_relabel_workspace_bytes(pr_ctx *ctx, int64_t N, int64_t E) {
  if (!ctx || bad_graph_sizes(N, E)) return 0;
  DeviceGuard g(ctx->device);
  size_t b = 0;
  return relabel_temp_bytes(N, E, &b) == hipSuccess ? b : 0;
}

int pr_relabel(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
               int64_t N, int64_t E, int32_t *perm, int32_t *out_offsets, int32_t *out_indices, int32_t *out_outdeg,
               void *workspace, size_t workspace_bytes) {
  if (!ctx || !in_offsets || !outdeg || !perm || !out_offsets || !out_outdeg || !workspace ||
      (E > 0 && (!in_indices || !out_indices))) {
    set_error("pr_relabel: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  DeviceGuard g(ctx->device);
  size_t need = 0;
  PR_HIP(relabel_temp_bytes(N, E, &need));
  if (workspace_bytes < need) {
    set_error("pr_relabel: workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return PR_ENOMEM;
  }
  PR_HIP(launch_relabel((hipStream_t)stream, in_offsets, in_indices, outdeg, (int32_t)N, (int32_t)E, perm,
                        out_offsets, out_indices, out_outdeg, workspace, workspace_bytes,
                        (uint32_t *)ctx->hscratch));
  return PR_OK;
}

int pr_unpermute(pr_ctx *ctx, void *stream, const int32_t *perm, int64_t N, const double *in, double *out) {
  if (!ctx || !perm || !in || !out) {
    set_error("pr_unpermute: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1 || N > 2147483646LL) {
    set_error("pr_unpermute: N must be in [1, 2^31-2], got %lld", (long long)N);
    return PR_EINVAL;
  }
  DeviceGuard g(ctx->device);
  PR_HIP(launch_unpermute((hipStream_t)stream, perm, (int32_t)N, in, out));
  return PR_OK;
}

size_t pr_workspace_bytes(int64_t N, int64_t E, int32_t precision, int32_t with_prep) {
  if (bad_graph_sizes(N, E) || (precision != PR_FP64 && precision != PR_MIXED && precision != PR_FP32)) return 0;
  return carve(nullptr, N, E, precision, with_prep != 0).total;
}

int pr_pull(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
            int64_t N, int64_t E, const void *prep, double alpha, double tau, int32_t norm, int32_t max_iter,
            int32_t precision, const double *init, double *ranks, double *norm_trace, void *workspace,
            size_t workspace_bytes, pr_result *out) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !workspace || !out || (E > 0 && !in_indices)) {
    set_error("pr_pull: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  if (!(alpha >= 0.0 && alpha <= 1.0)) {
    set_error("alpha must be in [0, 1], got %g", alpha);
    return PR_EINVAL;
  }
  if (!(tau >= 0.0)) {
    set_error("tau must be >= 0 and not NaN, got %g", tau);
    return PR_EINVAL;
  }
  if (norm < PR_L1 || norm > PR_LINF) {
    set_error("norm must be PR_L1, PR_L2 or PR_LINF, got %d", norm);
    return PR_EINVAL;
  }
  if (max_iter < 1) {
    set_error("max_iter must be >= 1, got %d", max_iter);
    return PR_EINVAL;
  }
  if (precision != PR_FP64 && precision != PR_MIXED && precision != PR_FP32) {
    set_error("precision must be PR_FP64, PR_MIXED or PR_FP32, got %d", precision);
    return PR_EINVAL;
  }
  const Layout L = carve(workspace, N, E, precision, prep == nullptr);
  if (workspace_bytes < L.total) {
    set_error("pr_pull: workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  int rc;
  const void *pp = prep;
  if (!prep) {
    rc = prepare_into(ctx, s, in_offsets, N, E, L.prep, &h);
    pp = L.prep;
  } else {
    rc = get_prep(ctx, s, prep, N, E, &h);
  }
  if (rc != PR_OK) return rc;

  PR_HIP(launch_fill_u32(s, (uint32_t *)L.st, sizeof(SolveState) / 4, 0u));
  const std::pair<int32_t, int64_t> ts = tuned_settings(ctx, h);
  const int64_t gcap = ts.second > 0 ? ts.second : ctx->resident[precision == PR_FP64 ? 0 : 1];
  const PrepPart &part = h.part[0];
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>({(int64_t)part.ndesc, gcap, kMaxGrid}));

  IterParams p{};
  p.off = in_offsets;
  p.idx = in_indices;
  p.outdeg = outdeg;
  p.desc = (const int4 *)((const char *)pp + part.desc_off);
  p.ndesc = part.ndesc;
  p.N = (int32_t)N;
  p.alpha = alpha;
  p.tau = tau;
  p.norm = norm;
  p.max_iter = max_iter;
  p.st = L.st;
  p.bpart = L.bpart;
  p.hpart = L.hpart;
  p.hubs = (const int4 *)((const char *)pp + part.hub_off);
  p.nhubs = part.nhubs;
  p.grid = (int32_t)grid;
  p.trace = norm_trace;
  p.mid_deg = ts.first;

  int fp32_iters = 0, fbuf = 0;
  const void *final_y = nullptr;
  bool final_fp32 = false;
  if (precision == PR_MIXED) {
    PR_HIP(launch_init(s, true, outdeg, (int32_t)N, init, L.y32[0], alpha, L.st, L.bpart, kMaxGrid));
    p.phase = 1;
    rc = run_until_stop(ctx, s, update_chunk(ctx, true, grid, p, L.y32[0], L.y32[1]), &L.st->head, max_iter, &fbuf);
    if (rc != PR_OK) return rc;
    fp32_iters = ((LoopHead *)ctx->hstate)->iter;
    if (((LoopHead *)ctx->hstate)->done) {
      final_y = L.y32[fbuf];
      final_fp32 = true;
    } else {
      PR_HIP(launch_convert(s, L.y32[fbuf], L.y64[0], (int32_t)N, L.st));
      p.phase = 2;
      rc = run_until_stop(ctx, s, update_chunk(ctx, false, grid, p, L.y64[0], L.y64[1]), &L.st->head, max_iter,
                          &fbuf);
      if (rc != PR_OK) return rc;
      final_y = L.y64[fbuf];
    }
  } else if (precision == PR_FP32) {
    // the float32 phase alone, stopping like a float64 solve (tau met or max_iter)
    PR_HIP(launch_init(s, true, outdeg, (int32_t)N, init, L.y32[0], alpha, L.st, L.bpart, kMaxGrid));
    p.phase = 0;
    rc = run_until_stop(ctx, s, update_chunk(ctx, true, grid, p, L.y32[0], L.y32[1]), &L.st->head, max_iter, &fbuf);
    if (rc != PR_OK) return rc;
    fp32_iters = ((LoopHead *)ctx->hstate)->iter;
    final_y = L.y32[fbuf];
    final_fp32 = true;
  } else {
    PR_HIP(launch_init(s, false, outdeg, (int32_t)N, init, L.y64[0], alpha, L.st, L.bpart, kMaxGrid));
    p.phase = 0;
    rc = run_until_stop(ctx, s, update_chunk(ctx, false, grid, p, L.y64[0], L.y64[1]), &L.st->head, max_iter, &fbuf);
    if (rc != PR_OK) return rc;
    final_y = L.y64[fbuf];
  }
  PR_HIP(launch_output(s, final_fp32, outdeg, final_y, (int32_t)N, ranks));
  PR_HIP(hipMemcpyAsync(ctx->hstate, L.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  const SolveState &hs = *ctx->hstate;
  out->iterations = hs.head.iter;
  out->converged = hs.converged;
  out->fp32_iters = precision == PR_FP64 ? 0 : fp32_iters;
  out->fp64_iters = hs.head.iter - out->fp32_iters;
  out->final_err[0] = hs.err[0];
  out->final_err[1] = hs.err[1];
  out->final_err[2] = hs.err[2];
  return hs.converged ? PR_OK : PR_NOT_CONVERGED;
}

size_t pr_batch_workspace_bytes(int64_t N, int64_t E, int32_t K, int32_t precision, int32_t with_prep) {
  if (bad_graph_sizes(N, E) || K < 1 || K > kMaxCols || (precision != PR_FP64 && precision != PR_MIXED)) return 0;
  return carve_batch(nullptr, N, E, K, precision, with_prep != 0).total;
}

int pr_pull_batch(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                  const int32_t *outdeg, int64_t N, int64_t E, const void *prep, int32_t K, const pr_problem *probs,
                  int32_t precision, const double *const *init, double *const *ranks, double *const *norm_trace,
                  void *workspace, size_t workspace_bytes, pr_result *results) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !probs || !workspace || !results || (E > 0 && !in_indices)) {
    set_error("pr_pull_batch: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  if (K < 1 || K > kMaxCols) {
    set_error("K must be in [1, %d], got %d", kMaxCols, K);
    return PR_EINVAL;
  }
  if (precision != PR_FP64 && precision != PR_MIXED) {
    set_error("precision must be PR_FP64 or PR_MIXED, got %d", precision);
    return PR_EINVAL;
  }
  for (int k = 0; k < K; ++k) {
    const pr_problem &q = probs[k];
    if (!(q.alpha >= 0.0 && q.alpha <= 1.0) || !(q.tau >= 0.0) || q.norm < PR_L1 || q.norm > PR_LINF ||
        q.max_iter < 1 || !ranks[k]) {
      set_error("problem %d: alpha in [0,1], tau >= 0, norm 1..3, max_iter >= 1 and a ranks buffer are required", k);
      return PR_EINVAL;
    }
  }
  const BatchLayout L = carve_batch(workspace, N, E, K, precision, prep == nullptr);
  if (workspace_bytes < L.total) {
    set_error("pr_pull_batch: workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  int rc;
  const void *pp = prep;
  if (!prep) {
    rc = prepare_into(ctx, s, in_offsets, N, E, L.prep, &h);
    pp = L.prep;
  } else {
    rc = get_prep(ctx, s, prep, N, E, &h);
  }
  if (rc != PR_OK) return rc;
  int max_iter = 1;
  for (int k = 0; k < K; ++k) max_iter = std::max(max_iter, probs[k].max_iter);

  const PrepPart &part = h.part[1];
  BatchParams p{};
  p.off = in_offsets;
  p.idx = in_indices;
  p.outdeg = outdeg;
  p.desc = (const int4 *)((const char *)pp + part.desc_off);
  p.ndesc = part.ndesc;
  p.N = (int32_t)N;
  p.nhubs = part.nhubs;
  p.hubs = (const int4 *)((const char *)pp + part.hub_off);
  p.bpart = L.bpart;
  p.hpart = L.hpart;
  p.hacc = L.hacc;
  p.st = L.st;
  p.cols = L.cols;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1) cus = 1;
  auto grid_of = [&](bool fp32, int kpw) {
    const int64_t res = ctx->max_grid > 0 ? ctx->max_grid : (int64_t)cus * batch_blocks_per_cu(fp32, kpw);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>({(int64_t)part.ndesc, res, kMaxGrid}));
  };

  // The running layout: slot i holds original problem orig[i]; `master` keeps every original
  // problem's latest column state on the host.
  int orig[kMaxCols];
  BatchColumn master[kMaxCols];
  memset(master, 0, sizeof master);
  int Kc = K;
  for (int i = 0; i < K; ++i) orig[i] = i;
  // Write the per-slot parameters (slot order) with the given map/ranks choice and wait for the
  // copy, so the pinned staging buffer may be rewritten afterwards.
  auto write_cols = [&](int n, const int *slot_orig, const int *map, bool with_ranks, const bool *rank_sel) -> int {
    BatchCols &hc = *ctx->hcols;
    memset(&hc, 0, sizeof hc);
    for (int i = 0; i < n; ++i) {
      const int k = slot_orig[i];
      hc.alpha[i] = probs[k].alpha;
      hc.tau[i] = probs[k].tau;
      hc.norm[i] = probs[k].norm;
      hc.max_iter[i] = probs[k].max_iter;
      hc.init[i] = init ? init[k] : nullptr;
      hc.ranks[i] = with_ranks && (!rank_sel || rank_sel[i]) ? ranks[k] : nullptr;
      hc.trace[i] = norm_trace ? norm_trace[k] : nullptr;
      hc.map[i] = map ? map[i] : -1;
    }
    PR_HIP(hipMemcpyAsync(L.cols, &hc, sizeof hc, hipMemcpyHostToDevice, s));
    PR_HIP(hipStreamSynchronize(s));
    return PR_OK;
  };
  auto stat_chunk = [&](const ChunkSpec &cs, const std::vector<hipEvent_t> *ev, int did) -> int {
    if (!ev || did <= 0) return PR_OK;
    float ms = 0.f;
    for (int k = 0; k < did && k < cs.count; ++k) {
      PR_HIP(hipEventElapsedTime(&ms, (*ev)[k], (*ev)[k + 1]));
      ctx->stat_ms[cs.kind] += ms;
      ctx->stat_launches[cs.kind] += 1;
      ctx->stat_ms[cs.sub_kind] += ms;
      ctx->stat_launches[cs.sub_kind] += 1;
    }
    return PR_OK;
  };

  const bool mixed = precision == PR_MIXED;
  const bool fp32 = mixed;  // first phase arithmetic
  const bool narrow = ctx->narrow != 0;
  int kp = batch_row_width(Kc, fp32, narrow);
  void *b0 = fp32 ? (void *)L.y32[0] : (void *)L.y64[0];
  void *b1 = fp32 ? (void *)L.y32[1] : (void *)L.y64[1];
  const int kp64 = batch_row_width(K, false, narrow);

  rc = write_cols(Kc, orig, nullptr, false, nullptr);
  if (rc != PR_OK) return rc;
  PR_HIP(launch_fill_u32(s, (uint32_t *)L.st, sizeof(BatchState) / 4, 0u));
  p.K = Kc;
  p.phase = mixed ? 1 : 0;
  p.grid = (int32_t)grid_of(fp32, kp);
  PR_HIP(launch_batch_init(s, fp32, outdeg, (int32_t)N, Kc, kp, b0, L.bpart, kMaxGrid, p, p.phase));

  // ---- first phase, with compaction of the active columns into narrower rows
  int before = 0;
  for (int rounds = 0;; ++rounds) {
    ChunkSpec cs = batch_chunk(ctx, fp32, kp, (unsigned)p.grid, p, b0, b1);
    cs.count = (int)ctx->batch_chunk;
    const std::vector<hipEvent_t> *ev = nullptr;
    rc = run_chunk(ctx, s, cs, &ev);
    if (rc != PR_OK) return rc;
    PR_HIP(hipMemcpyAsync(ctx->hbstate, L.st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
    PR_HIP(hipStreamSynchronize(s));
    BatchState &hs = *ctx->hbstate;
    rc = stat_chunk(cs, ev, hs.head.phase_iter - before);
    if (rc != PR_OK) return rc;
    before = hs.head.phase_iter;
    for (int i = 0; i < Kc; ++i) master[orig[i]] = hs.col[i];
    if (hs.head.stop) break;
    if (rounds > max_iter + 2) {
      set_error("internal: update limit passed without stop");
      return PR_EDEVICE;
    }
    int act[kMaxCols], nact = 0;
    bool leaving[kMaxCols];
    for (int i = 0; i < Kc; ++i) {
      leaving[i] = !hs.col[i].active;
      if (hs.col[i].active) act[nact++] = i;
    }
    const int kp2 = batch_row_width(nact, fp32, narrow);
    if (ctx->compact == 0 || nact == Kc || kp2 >= kp) continue;
    // (a) columns leaving the layout: float32 -> their float64 columns (mixed), or final ranks
    if (mixed) {
      int map[kMaxCols];
      for (int i = 0; i < Kc; ++i) map[i] = leaving[i] ? orig[i] : -1;
      rc = write_cols(Kc, orig, map, false, nullptr);
      if (rc != PR_OK) return rc;
      PR_HIP(launch_batch_convert(s, (const float *)b0, (const float *)b1, kp, L.y64[0], kp64, (int32_t)N, Kc, L.st,
                                  L.cols));
    } else {
      rc = write_cols(Kc, orig, nullptr, true, leaving);
      if (rc != PR_OK) return rc;
      p.K = Kc;
      PR_HIP(launch_batch_output(s, false, outdeg, b0, b1, kp, (int32_t)N, Kc, p));
    }
    // (b) repack the active columns (all at the same parity) into the other buffer
    const int par = hs.col[act[0]].phase_updates & 1;
    void *cur = par ? b1 : b0, *oth = par ? b0 : b1;
    int norig[kMaxCols];
    for (int i = 0; i < nact; ++i) norig[i] = orig[act[i]];
    rc = write_cols(nact, norig, act, false, nullptr);
    if (rc != PR_OK) return rc;
    PR_HIP(launch_batch_compact(s, fp32, cur, kp, oth, kp2, (int32_t)N, nact, L.cols));
    // (c) the slot states follow their columns; the repacked buffer becomes buffer 0
    BatchState ns = hs;
    for (int i = 0; i < kMaxCols; ++i) {
      if (i < nact) {
        ns.col[i] = hs.col[act[i]];
        ns.col[i].phase_updates = 0;
      } else {
        memset(&ns.col[i], 0, sizeof ns.col[i]);
        ns.col[i].done = 1;
      }
    }
    hs = ns;
    PR_HIP(hipMemcpyAsync(L.st, &hs, sizeof(BatchState), hipMemcpyHostToDevice, s));
    PR_HIP(hipStreamSynchronize(s));
    Kc = nact;
    for (int i = 0; i < nact; ++i) orig[i] = norig[i];
    kp = kp2;
    b0 = oth;
    b1 = cur;
    p.K = Kc;
    p.grid = (int32_t)grid_of(fp32, kp);
    before = 0;
    hs.head.phase_iter = 0;
    PR_HIP(launch_fill_u32(s, (uint32_t *)&L.st->head.phase_iter, 1, 0u));
  }

  const BatchColumn *fin = master;
  if (mixed) {
    // remaining float32 columns -> float64, then the float64 phase over all K problems
    int map[kMaxCols];
    for (int i = 0; i < Kc; ++i) map[i] = orig[i];
    rc = write_cols(Kc, orig, map, false, nullptr);
    if (rc != PR_OK) return rc;
    PR_HIP(launch_batch_convert(s, (const float *)b0, (const float *)b1, kp, L.y64[0], kp64, (int32_t)N, Kc, L.st,
                                L.cols));
    int all[kMaxCols];
    for (int i = 0; i < K; ++i) all[i] = i;
    rc = write_cols(K, all, nullptr, true, nullptr);
    if (rc != PR_OK) return rc;
    BatchState &hs = *ctx->hbstate;
    memset(&hs, 0, sizeof hs);
    for (int i = 0; i < kMaxCols; ++i) {
      if (i < K) {
        hs.col[i] = master[i];
      } else {
        hs.col[i].done = 1;
      }
    }
    hs.phase = 2;
    PR_HIP(hipMemcpyAsync(L.st, &hs, sizeof(BatchState), hipMemcpyHostToDevice, s));
    PR_HIP(hipStreamSynchronize(s));
    PR_HIP(launch_batch_rearm(s, L.st, K));
    p.K = K;
    p.phase = 2;
    p.grid = (int32_t)grid_of(false, kp64);
    int fbuf = 0;
    rc = run_until_stop(ctx, s, batch_chunk(ctx, false, kp64, (unsigned)p.grid, p, L.y64[0], L.y64[1]), &L.st->head,
                        max_iter, &fbuf);
    if (rc != PR_OK) return rc;
    PR_HIP(launch_batch_output(s, false, outdeg, L.y64[0], L.y64[1], kp64, (int32_t)N, K, p));
    PR_HIP(hipMemcpyAsync(ctx->hbstate, L.st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
    PR_HIP(hipStreamSynchronize(s));
    fin = ctx->hbstate->col;
  } else {
    rc = write_cols(Kc, orig, nullptr, true, nullptr);
    if (rc != PR_OK) return rc;
    p.K = Kc;
    PR_HIP(launch_batch_output(s, false, outdeg, b0, b1, kp, (int32_t)N, Kc, p));
    PR_HIP(hipStreamSynchronize(s));
  }
  int all_conv = 1;
  for (int k = 0; k < K; ++k) {
    const BatchColumn &c = fin[k];
    results[k].iterations = c.iters;
    results[k].converged = c.converged;
    results[k].fp32_iters = c.fp32_iters;
    results[k].fp64_iters = c.iters - c.fp32_iters;
    results[k].final_err[0] = c.err[0];
    results[k].final_err[1] = c.err[1];
    results[k].final_err[2] = c.err[2];
    all_conv &= c.converged;
  }
  return all_conv ? PR_OK : PR_NOT_CONVERGED;
}

int pr_l1_distance(pr_ctx *ctx, void *stream, const double *x, const double *y, int64_t N, void *workspace,
                   size_t workspace_bytes, double *out) {
  if (!ctx || !x || !y || !workspace || !out) {
    set_error("pr_l1_distance: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1) {
    set_error("pr_l1_distance: N must be >= 1");
    return PR_EINVAL;
  }
  constexpr int32_t nb = 1024;
  if (workspace_bytes < (nb + 1) * sizeof(double)) {
    set_error("pr_l1_distance: workspace needs %zu bytes", (size_t)(nb + 1) * sizeof(double));
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  double *part = (double *)workspace;
  PR_HIP(launch_l1(s, x, y, N, part, nb));
  PR_HIP(hipMemcpyAsync(ctx->hscratch, part + nb, sizeof(double), hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  memcpy(out, ctx->hscratch, sizeof(double));
  return PR_OK;
}

static size_t multi_layout(int32_t G, const pr_graph_problem *probs, void *ws, MultiGraph **graphs,
                           MultiGraphState **states, int32_t **tile_base, double **part, GridBarrier **bar,
                           double **hpart, double **y, void **preps) {
  Carver c(ws);
  *bar = (GridBarrier *)c.take(sizeof(GridBarrier));
  *graphs = (MultiGraph *)c.take(sizeof(MultiGraph) * (size_t)G);
  *states = (MultiGraphState *)c.take(sizeof(MultiGraphState) * (size_t)G);
  *tile_base = (int32_t *)c.take(sizeof(int32_t) * (size_t)(G + 1));
  *part = (double *)c.take(sizeof(double) * 4 * (size_t)kMaxGrid * (size_t)G);
  for (int g = 0; g < G; ++g) {
    hpart[g] = (double *)c.take(sizeof(double) * (size_t)max_slots(probs[g].N, probs[g].E));
    y[2 * g] = (double *)c.take(sizeof(double) * (size_t)probs[g].N);
    y[2 * g + 1] = (double *)c.take(sizeof(double) * (size_t)probs[g].N);
    preps[g] = probs[g].prep ? nullptr : c.take(prep_bytes(probs[g].N, probs[g].E));
  }
  return c.used;
}

size_t pr_multi_workspace_bytes(int32_t G, const pr_graph_problem *probs) {
  if (G < 1 || G > kMaxGraphs || !probs) return 0;
  for (int g = 0; g < G; ++g)
    if (bad_graph_sizes(probs[g].N, probs[g].E)) return 0;
  MultiGraph *a;
  MultiGraphState *b;
  int32_t *c;
  double *d;
  GridBarrier *e;
  std::vector<double *> hp(G), y(2 * G);
  std::vector<void *> pp(G);
  return multi_layout(G, probs, nullptr, &a, &b, &c, &d, &e, hp.data(), y.data(), pp.data());
}

int pr_pull_multi(pr_ctx *ctx, void *stream, int32_t G, const pr_graph_problem *probs, void *workspace,
                  size_t workspace_bytes, pr_result *results) {
  if (!ctx || !probs || !workspace || !results) {
    set_error("pr_pull_multi: NULL argument");
    return PR_EINVAL;
  }
  if (G < 1 || G > kMaxGraphs) {
    set_error("G must be in [1, %d], got %d", kMaxGraphs, G);
    return PR_EINVAL;
  }
  int max_rounds = 1;
  int64_t total_tiles = 0;
  for (int g = 0; g < G; ++g) {
    const pr_graph_problem &q = probs[g];
    if (!q.in_offsets || !q.outdeg || !q.ranks || (q.E > 0 && !q.in_indices)) {
      set_error("graph %d: NULL graph or ranks pointer", g);
      return PR_EINVAL;
    }
    if (bad_graph_sizes(q.N, q.E)) return PR_EINVAL;
    if (!(q.alpha >= 0.0 && q.alpha <= 1.0) || !(q.tau >= 0.0) || q.norm < PR_L1 || q.norm > PR_LINF ||
        q.max_iter < 1) {
      set_error("graph %d: alpha in [0,1], tau >= 0, norm 1..3 and max_iter >= 1 are required", g);
      return PR_EINVAL;
    }
    max_rounds = std::max(max_rounds, q.max_iter);
  }
  MultiGraph *dgraphs;
  MultiGraphState *dstates;
  int32_t *dbase;
  double *dpart;
  GridBarrier *dbar;
  std::vector<double *> hpart(G), ybuf(2 * G);
  std::vector<void *> ownprep(G);
  const size_t need = multi_layout(G, probs, workspace, &dgraphs, &dstates, &dbase, &dpart, &dbar, hpart.data(),
                                   ybuf.data(), ownprep.data());
  if (workspace_bytes < need) {
    set_error("pr_pull_multi: workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return PR_ENOMEM;
  }
  DeviceGuard dg(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  std::vector<MultiGraph> hg(G);
  std::vector<int32_t> base(G + 1, 0);
  for (int g = 0; g < G; ++g) {
    const pr_graph_problem &q = probs[g];
    PrepHeader h;
    int rc;
    const void *pp = q.prep;
    if (!pp) {
      rc = prepare_into(ctx, s, q.in_offsets, q.N, q.E, ownprep[g], &h);
      pp = ownprep[g];
    } else {
      rc = get_prep(ctx, s, pp, q.N, q.E, &h);
    }
    if (rc != PR_OK) return rc;
    const PrepPart &part = h.part[0];
    MultiGraph &m = hg[g];
    memset(&m, 0, sizeof m);
    m.off = q.in_offsets;
    m.idx = q.in_indices;
    m.outdeg = q.outdeg;
    m.desc = (const int4 *)((const char *)pp + part.desc_off);
    m.hubs = (const int4 *)((const char *)pp + part.hub_off);
    m.nhubs = part.nhubs;
    m.hpart = hpart[g];
    m.y[0] = ybuf[2 * g];
    m.y[1] = ybuf[2 * g + 1];
    m.init = q.init;
    m.ranks = q.ranks;
    m.trace = q.norm_trace;
    m.alpha = q.alpha;
    m.tau = q.tau;
    m.N = (int32_t)q.N;
    m.norm = q.norm;
    m.max_iter = q.max_iter;
    m.mid_deg = tuned_settings(ctx, h).first;
    total_tiles += part.ndesc;
    if (total_tiles > 2147483647LL) {
      set_error("pr_pull_multi: more than 2^31 tiles in one batch");
      return PR_EINVAL;
    }
    base[g + 1] = (int32_t)total_tiles;
  }
  // stage the tables through pinned memory (synchronised before the buffer is reused)
  const size_t tbytes = sizeof(MultiGraph) * (size_t)G + sizeof(int32_t) * (size_t)(G + 1);
  if (ctx->hmulti_bytes < tbytes) {
    if (ctx->hmulti) (void)hipHostFree(ctx->hmulti);
    ctx->hmulti = nullptr;
    ctx->hmulti_bytes = 0;
    PR_HIP(hipHostMalloc(&ctx->hmulti, tbytes, hipHostMallocDefault));
    ctx->hmulti_bytes = tbytes;
  }
  char *hm = (char *)ctx->hmulti;
  memcpy(hm, hg.data(), sizeof(MultiGraph) * (size_t)G);
  memcpy(hm + sizeof(MultiGraph) * (size_t)G, base.data(), sizeof(int32_t) * (size_t)(G + 1));
  PR_HIP(hipMemcpyAsync(dgraphs, hm, sizeof(MultiGraph) * (size_t)G, hipMemcpyHostToDevice, s));
  PR_HIP(hipMemcpyAsync(dbase, hm + sizeof(MultiGraph) * (size_t)G, sizeof(int32_t) * (size_t)(G + 1),
                        hipMemcpyHostToDevice, s));
  MultiParams p{};
  p.graphs = dgraphs;
  p.states = dstates;
  p.tile_base = dbase;
  p.part = dpart;
  p.bar = dbar;
  {
    int khz = 0;  // wall clock of the device (s_memrealtime), 100 MHz on this GPU family
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz < 1)
      khz = 100000;
    p.wait_ticks = (uint64_t)ctx->barrier_ms * (uint64_t)khz;
  }
  p.G = G;
  p.total_tiles = (int32_t)total_tiles;
  p.max_rounds = max_rounds;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1) cus = 1;
  const int64_t resident = (int64_t)cus * multi_blocks_per_cu();
  int64_t grid = ctx->max_grid > 0 ? std::min<int64_t>(ctx->max_grid, resident) : resident;
  grid = std::max<int64_t>(1, std::min<int64_t>({grid, total_tiles > 0 ? total_tiles : 1, (int64_t)kMaxGrid}));
  EventPair ev;  // destroyed on every return
  if (ctx->timing) {
    PR_HIP(hipEventCreate(&ev.a));
    PR_HIP(hipEventCreate(&ev.b));
    PR_HIP(hipEventRecord(ev.a, s));
  }
  PR_HIP(launch_fill_u32(s, (uint32_t *)dbar, sizeof(GridBarrier) / 4, 0u));
  PR_HIP(launch_multi(s, (unsigned)grid, p, 64));
  if (ctx->timing) PR_HIP(hipEventRecord(ev.b, s));
  std::vector<MultiGraphState> hs(G);
  uint32_t timed_out = 0;
  PR_HIP(hipMemcpyAsync(ctx->hmulti, dstates, sizeof(MultiGraphState) * (size_t)G, hipMemcpyDeviceToHost, s));
  PR_HIP(hipMemcpyAsync((char *)ctx->hmulti + sizeof(MultiGraphState) * (size_t)G, &dbar->timeout[0],
                        sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  memcpy(hs.data(), ctx->hmulti, sizeof(MultiGraphState) * (size_t)G);
  memcpy(&timed_out, (char *)ctx->hmulti + sizeof(MultiGraphState) * (size_t)G, sizeof(uint32_t));
  if (ctx->timing) {
    float ms = 0.f;
    PR_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    ctx->stat_ms[PR_KERNEL_MULTI] += ms;
    ctx->stat_launches[PR_KERNEL_MULTI] += 1;
  }
  if (timed_out) {
    set_error("pr_pull_multi: a grid barrier wait of the launch passed its time limit");
    return PR_EDEVICE;
  }
  int all = 1;
  for (int g = 0; g < G; ++g) {
    results[g].iterations = hs[g].iters;
    results[g].converged = hs[g].converged;
    results[g].fp32_iters = 0;
    results[g].fp64_iters = hs[g].iters;
    results[g].final_err[0] = hs[g].err[0];
    results[g].final_err[1] = hs[g].err[1];
    results[g].final_err[2] = hs[g].err[2];
    all &= hs[g].converged;
  }
  return all ? PR_OK : PR_NOT_CONVERGED;
}

int pr_autotune(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                const int32_t *outdeg, int64_t N, int64_t E, const void *prep, double *ranks, void *workspace,
                size_t workspace_bytes, pr_tune_result *out) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !workspace || !out || (E > 0 && !in_indices)) {
    set_error("pr_autotune: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  const Layout L = carve(workspace, N, E, PR_FP64, prep == nullptr);
  if (workspace_bytes < L.total) {
    set_error("pr_autotune: workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    return PR_ENOMEM;
  }
  const void *pp = prep;
  int rc;
  if (!prep) {
    rc = prepare_into(ctx, s, in_offsets, N, E, L.prep, &h);
    pp = L.prep;
  } else {
    rc = get_prep(ctx, s, prep, N, E, &h);
  }
  if (rc != PR_OK) return rc;
  // candidates: lane/wave threshold x update grid (in resident workgroups)
  const int32_t mids[] = {8, 16, 32, 64, 128};
  const int64_t res = ctx->resident[0];
  const int64_t grids[] = {res, 2 * res, 4 * res};
  const int64_t save_grid = ctx->max_grid, save_mid = ctx->mid_deg, save_timing = ctx->timing;
  const bool save_set = ctx->mid_deg_set;
  const int64_t save_tuned = ctx->use_tuned;
  int64_t save_launch[PR_KERNEL_KINDS];
  double save_ms[PR_KERNEL_KINDS];
  memcpy(save_launch, ctx->stat_launches, sizeof save_launch);
  memcpy(save_ms, ctx->stat_ms, sizeof save_ms);
  ctx->use_tuned = 0;
  ctx->mid_deg_set = true;
  ctx->timing = 1;
  double best = 1e300, dflt = 0.0;
  int32_t best_mid = kMidDeg, best_grid = (int32_t)std::min<int64_t>(res, kMaxGrid);
  int count = 0;
  constexpr int kReps = 4;
  for (int64_t gsz : grids) {
    if (gsz > kMaxGrid) continue;
    for (int32_t m : mids) {
      ctx->max_grid = gsz;
      ctx->mid_deg = m;
      ctx->stat_launches[PR_KERNEL_UPDATE_F64] = 0;
      ctx->stat_ms[PR_KERNEL_UPDATE_F64] = 0.0;
      pr_result r;
      rc = pr_pull(ctx, stream, in_offsets, in_indices, outdeg, N, E, pp, 0.85, 0.0, PR_L1, kReps, PR_FP64, nullptr,
                   ranks, nullptr, workspace, workspace_bytes, &r);
      if (rc < 0) break;
      const double us = ctx->stat_launches[PR_KERNEL_UPDATE_F64]
                            ? 1e3 * ctx->stat_ms[PR_KERNEL_UPDATE_F64] / ctx->stat_launches[PR_KERNEL_UPDATE_F64]
                            : 1e300;
      ++count;
      if (gsz == res && m == kMidDeg) dflt = us;
      if (us < best) {
        best = us;
        best_mid = m;
        best_grid = (int32_t)gsz;
      }
    }
    if (rc < 0) break;
  }
  ctx->max_grid = save_grid;
  ctx->mid_deg = save_mid;
  ctx->mid_deg_set = save_set;
  ctx->timing = save_timing;
  ctx->use_tuned = save_tuned;
  memcpy(ctx->stat_launches, save_launch, sizeof save_launch);
  memcpy(ctx->stat_ms, save_ms, sizeof save_ms);
  if (rc < 0) return rc;
  const std::vector<int64_t> sig = graph_signature(h);
  ctx->tuned[sig] = {best_mid, best_grid};
  save_tune_entry(ctx, sig, best_mid, best_grid);
  out->mid_deg = best_mid;
  out->grid = best_grid;
  out->candidates = count;
  out->pad = 0;
  out->best_us = best;
  out->default_us = dflt;
  return PR_OK;
}

int pr_mlp_param_count(void) { return mlp_param_count(); }

int pr_features(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
                int64_t N, int64_t E, const void *prep, const double *r085, double alpha_target, float *feat,
                const double *r_target, float *target) {
  if (!ctx || !in_offsets || !outdeg || !prep || !r085 || !feat || (E > 0 && !in_indices) ||
      ((r_target == nullptr) != (target == nullptr))) {
    set_error("pr_features: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  const int rc = get_prep(ctx, s, prep, N, E, &h);
  if (rc != PR_OK) return rc;
  const PrepPart &part = h.part[0];
  PR_HIP(launch_features(s, in_offsets, in_indices, outdeg, (int32_t)N,
                         (const int4 *)((const char *)prep + part.desc_off), part.ndesc,
                         (const int4 *)((const char *)prep + part.hub_off), part.nhubs, r085, alpha_target, feat,
                         r_target, target));
  return PR_OK;
}

int pr_mlp_forward(pr_ctx *ctx, void *stream, const float *W, const float *feat, int64_t N, float *y,
                   uint16_t *act_save) {
  if (!ctx || !W || !feat || !y) {
    set_error("pr_mlp_forward: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1) {
    set_error("pr_mlp_forward: N must be >= 1");
    return PR_EINVAL;
  }
  if (((uintptr_t)act_save & 7) != 0) {
    set_error("pr_mlp_forward: act_save must be 8-byte aligned");
    return PR_EINVAL;
  }
  DeviceGuard g(ctx->device);
  PR_HIP(launch_mlp_forward((hipStream_t)stream, W, feat, N, y, act_save));
  return PR_OK;
}

size_t pr_mlp_backward_workspace_bytes(int64_t N) {
  if (N < 1 || N > 2147483646LL) return 0;
  const int nb = mlp_backward_blocks(N);
  return align_up(sizeof(float) * (size_t)nb * (size_t)mlp_param_count(), 256) +
         align_up(sizeof(double) * (size_t)(nb + 1), 256);
}

int pr_mlp_backward(pr_ctx *ctx, void *stream, const float *W, const float *feat, const uint16_t *act_save,
                    const float *y, const float *target, int64_t N, float *dW, void *workspace, size_t workspace_bytes,
                    double *loss) {
  if (!ctx || !W || !feat || !act_save || !y || !target || !dW || !workspace || !loss) {
    set_error("pr_mlp_backward: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1) {
    set_error("pr_mlp_backward: N must be >= 1");
    return PR_EINVAL;
  }
  if (((uintptr_t)act_save & 7) != 0) {
    set_error("pr_mlp_backward: act_save must be 8-byte aligned");
    return PR_EINVAL;
  }
  if (workspace_bytes < pr_mlp_backward_workspace_bytes(N)) {
    set_error("pr_mlp_backward: workspace has %zu bytes, needs %zu", workspace_bytes,
              pr_mlp_backward_workspace_bytes(N));
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const int nb = mlp_backward_blocks(N);
  float *part = (float *)workspace;
  double *lpart = (double *)((char *)workspace + align_up(sizeof(float) * (size_t)nb * (size_t)mlp_param_count(), 256));
  PR_HIP(launch_mlp_backward(s, W, feat, act_save, y, target, N, part, lpart, dW, lpart + nb));
  PR_HIP(hipMemcpyAsync(ctx->hscratch, lpart + nb, sizeof(double), hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  memcpy(loss, ctx->hscratch, sizeof(double));
  return PR_OK;
}

int pr_adam_step(pr_ctx *ctx, void *stream, float *W, const float *dW, float *m, float *v, int32_t n_params, float lr,
                 float beta1, float beta2, float eps, int32_t step) {
  if (!ctx || !W || !dW || !m || !v || n_params < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f)) {
    set_error("pr_adam_step: bad argument");
    return PR_EINVAL;
  }
  DeviceGuard g(ctx->device);
  PR_HIP(launch_adam((hipStream_t)stream, W, dW, m, v, n_params, lr, beta1, beta2, eps, step));
  return PR_OK;
}

int pr_warm_start_vector(pr_ctx *ctx, void *stream, const float *feat, const float *y, int64_t N, double *r0,
                         void *workspace, size_t workspace_bytes) {
  if (!ctx || !feat || !y || !r0 || !workspace) {
    set_error("pr_warm_start_vector: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1) {
    set_error("pr_warm_start_vector: N must be >= 1");
    return PR_EINVAL;
  }
  if (workspace_bytes < 1024 * sizeof(double)) {
    set_error("pr_warm_start_vector: workspace needs 8192 bytes");
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  PR_HIP(launch_start_vector((hipStream_t)stream, feat, y, N, r0, (double *)workspace));
  return PR_OK;
}

}  // extern "C"
