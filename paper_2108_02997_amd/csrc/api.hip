// api.hip -- the C ABI of libprpull.so (declared in include/prpull.h): argument checks,
// workspace carving, graph prep caching and the on-device-convergence iteration loop.
//
// The loop: updates are launched in chunks of `chunk` kernels, alternating the two iterate
// buffers.  A chunk is captured once into a HIP graph (on a private capture stream) and
// replayed on the caller's stream; once an update meets the stopping rule the remaining
// kernels of the chunk return at entry.  After each chunk the host reads the 64-byte solve
// state from pinned memory and stops when the device says so.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "api_internal.h"

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

Layout carve(void *ws, int64_t N, int64_t E, int32_t precision, bool with_prep) {
  Carver c(ws);
  Layout L{};
  L.st = (SolveState *)c.take(sizeof(SolveState));
  L.bpart = (double *)c.take(4 * sizeof(double) * (size_t)kMaxGrid);
  const int64_t slots = max_slots(N, E);
  L.hpart = (double *)c.take(sizeof(double) * (size_t)slots);
  L.snap = (SnapTable *)c.take(sizeof(SnapTable));
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
  h.version = kPrepVersion;
  h.N = N;
  h.E = E;
  h.seg = kSeg;
  return prepare_parts(ctx, s, off, N, E, prep, (int)ctx->window_tile[0], (int)ctx->window_tile[1], &h, out);
}

// Partitions A and B of `prep` with the given tile windows (rows = tile / 2) into header h (its
// other fields kept), header written and remembered.
int prepare_parts(pr_ctx *ctx, hipStream_t s, const int32_t *off, int64_t N, int64_t E, void *prep, int tile_a,
                  int tile_b, PrepHeader *hin, PrepHeader *out) {
  PrepHeader h = *hin;
  const int tiles[2] = {tile_a, tile_b};
  int64_t o = (int64_t)align_up(sizeof(PrepHeader), 256);
  for (int i = 0; i < 2; ++i) {
    PrepPart &pp = h.part[i];
    pp.tile = tiles[i];
    pp.rows = tiles[i] / 2;
    if (!valid_window(i, pp.tile, pp.rows)) {
      set_error("internal: tile window %d/%d not available for partition %d", pp.tile, pp.rows, i);
      return PR_EINVAL;
    }
    pp.desc_off = o;
    o += (int64_t)align_up((size_t)(max_desc(N, E, kMinPartTile[i], kMinPartRows[i]) + 1) * sizeof(int4), 256);
    pp.hub_off = o;
    o += (int64_t)align_up((size_t)max_hubs(N, E) * sizeof(int4), 256);
  }
  h.scan_off = o;
  char *base = (char *)prep;
  for (int i = 0; i < 2; ++i) {
    PrepPart &pp = h.part[i];
    PR_HIP(launch_prepare(s, pp.tile, pp.rows, off, N, (int4 *)(base + pp.desc_off), (int4 *)(base + pp.hub_off),
                          base + h.scan_off, ctx->hscratch));
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
  *hin = h;
  int rc = write_prep_header(ctx, s, prep, h);
  if (rc != PR_OK) return rc;
  *out = h;
  return PR_OK;
}

// The header to the device (synchronised) and into the context's table of preps.
int write_prep_header(pr_ctx *ctx, hipStream_t s, void *prep, const PrepHeader &h) {
  static_assert(sizeof(PrepHeader) <= 56 * sizeof(unsigned long long), "header staging");
  memcpy(ctx->hscratch + 8, &h, sizeof h);
  PR_HIP(hipMemcpyAsync(prep, ctx->hscratch + 8, sizeof h, hipMemcpyHostToDevice, s));
  PR_HIP(hipStreamSynchronize(s));
  ctx->preps[prep] = h;
  return PR_OK;
}

// Key bits of the segment sort: enough for every segment id of N sources (at least 1); with
// seg_len 1, for every source id.
int seg_key_bits(int64_t N, int32_t seg_len) {
  const int64_t S = (N - 1) / seg_len + 1;
  int k = 1;
  while (k < 31 && ((int64_t)1 << k) < S) ++k;
  return k;
}

// Layout of the source-segmented part of a prep buffer with P pairs, after the plain prep;
// false when a hipCUB size query fails.
bool seg_layout(int64_t N, int64_t E, int32_t seg_len, int64_t P, SegLayout *sl) {
  size_t sort_b = 0, scan_e = 0, scan_p = 0, tile_b = 0;
  if (seg_sort_temp_bytes(P, seg_key_bits(N, seg_len), &sort_b) != hipSuccess ||
      seg_scan_temp_bytes(E + 1, &scan_e) != hipSuccess || seg_scan_temp_bytes(P + 1, &scan_p) != hipSuccess ||
      seg_tile_sort_temp_bytes(E, max_desc(P, E, kPairTile, kRows), seg_key_bits(N, 1), &tile_b) != hipSuccess)
    return false;
  SegLayout L{};
  L.pairs = P;
  size_t o = align_up(prep_bytes(N, E), 256);
  auto take = [&o](size_t n) {
    const size_t at = o;
    o += align_up(n, 256);
    return (int64_t)at;
  };
  L.poff_off = take(4 * (size_t)(P + 1));
  L.moff_off = take(4 * (size_t)(N + 1));
  L.mpos_off = take(4 * (size_t)P);
  L.sidx_off = take(4 * (size_t)(E + 1));
  L.part_off = take(8 * (size_t)P);
  L.pair_part.tile = kPairTile;
  L.pair_part.rows = kRows;
  L.pair_part.desc_off = take((size_t)(max_desc(P, E, kPairTile, kRows) + 1) * sizeof(int4));
  L.pair_part.hub_off = take((size_t)max_hubs(P, E) * sizeof(int4));
  L.merge_part.tile = kTile;
  L.merge_part.rows = kRows;
  L.merge_part.desc_off = take((size_t)(max_desc(N, P, kTile, kRows) + 1) * sizeof(int4));
  L.merge_part.hub_off = take((size_t)max_hubs(N, P) * sizeof(int4));
  L.scan_off = take((size_t)(scan_block_count(std::max<int64_t>(N, P)) + 1) * 2 * sizeof(unsigned long long));
  L.temp_off = take(4 * (size_t)(E + 1));
  const size_t tail = o;
  take(4 * (size_t)(P + 1));
  take(4 * (size_t)(P + 1));
  take(4 * (size_t)P);
  // hipCUB's storage; first the pair count's block sums
  L.cub_off = take(std::max({sort_b, scan_e, scan_p, (size_t)(seg_count_blocks() + 1) * sizeof(unsigned long long)}));
  // the tiles' sort runs after the build and reuses the scratch behind temp
  const size_t tiles = (size_t)max_desc(P, E, kPairTile, kRows);
  const size_t tsort = seg_tile_sort_scratch(E, (int64_t)tiles, tile_b);
  L.tsort_off = (int64_t)tail;
  o = std::max(o, tail + tsort);
  L.tsort_bytes = (int64_t)(o - tail);
  L.total = (int64_t)o;
  *sl = L;
  return true;
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
  if (h.magic != kPrepMagic || h.version != kPrepVersion) {
    set_error("prep buffer was not written by pr_prepare");
    return PR_EINVAL;
  }
  if (h.N != N || h.E != E || h.seg != kSeg || !valid_window(0, h.part[0].tile, h.part[0].rows) ||
      !valid_window(1, h.part[1].tile, h.part[1].rows)) {
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
    r.node = k;
    const hipError_t e = launch_update(s, fp32, grid, r);
    if (e != hipSuccess || !r.snap) return e;
    return launch_snap(s, fp32, r);
  };
  return c;
}

// Row width (values per vertex) of the batch state for K columns: 1 or 2 (narrow rows, one lane
// per row fetch), else 4 * ceil(K / 4) = 4, 8, 12 or 16, in either precision (a random 48-byte
// float32 row costs less than a 64-byte one, so 9 to 12 columns are not padded to 16).
int batch_row_width(int K, bool fp32, bool narrow) {
  (void)fp32;
  if (narrow && K <= 2) return K < 1 ? 1 : K;
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
  return {h.N, h.E, h.part[0].ndesc, h.part[0].nhubs, h.part[0].nslots, h.part[1].ndesc, h.part[0].tile,
          h.part[1].tile};
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

// Key of the segmented-update settings: the graph signature and the layout's segment length.
std::vector<int64_t> seg_signature(const PrepHeader &h) {
  std::vector<int64_t> s = graph_signature(h);
  s.push_back(h.seg_len);
  return s;
}

// (wave-per-row threshold, workgroups per resident slot) of pr_pull_batch for a graph: the
// autotuner's table, else the defaults.
std::pair<int32_t, int32_t> tuned_batch_settings(pr_ctx *ctx, const PrepHeader &h) {
  if (ctx->use_tuned) {
    auto it = ctx->tuned_batch.find(graph_signature(h));
    if (it != ctx->tuned_batch.end()) return it->second;
  }
  return {kMidDeg, 1};
}

// Tune file lines: the graph signature (8 numbers), then mid_deg, grid, batch mid_deg, batch
// workgroups per resident slot; or "seg", the graph signature, the segment length, then the
// segmented update's pair threshold, per-segment grid and merge tile order.  Other lines are
// skipped.
void load_tune_file(pr_ctx *ctx) {
  const char *f = getenv("PRPULL_TUNE_FILE");
  if (!f || !*f) return;
  ctx->tune_file = f;
  FILE *fp = fopen(f, "r");
  if (!fp) return;
  char line[512];
  while (fgets(line, sizeof line, fp)) {
    long long s[9];
    int m, g, mb, gb;
    if (sscanf(line, "seg %lld %lld %lld %lld %lld %lld %lld %lld %lld %d %d %d", &s[0], &s[1], &s[2], &s[3], &s[4],
               &s[5], &s[6], &s[7], &s[8], &m, &g, &mb) == 12) {
      ctx->tuned_seg[std::vector<int64_t>(s, s + 9)] = SegTune{m, g, mb};
    } else if (sscanf(line, "%lld %lld %lld %lld %lld %lld %lld %lld %d %d %d %d", &s[0], &s[1], &s[2], &s[3], &s[4],
                      &s[5], &s[6], &s[7], &m, &g, &mb, &gb) == 12) {
      const std::vector<int64_t> sig(s, s + 8);
      ctx->tuned[sig] = {m, g};
      ctx->tuned_batch[sig] = {mb, gb};
    }
  }
  fclose(fp);
}

void save_tune_seg_entry(pr_ctx *ctx, const std::vector<int64_t> &sig, const SegTune &t) {
  if (ctx->tune_file.empty()) return;
  FILE *fp = fopen(ctx->tune_file.c_str(), "a");
  if (!fp) return;
  fprintf(fp, "seg");
  for (int64_t x : sig) fprintf(fp, " %lld", (long long)x);
  fprintf(fp, " %d %d %d\n", t.pair_mid_deg, t.seg_grid, t.merge_xcd);
  fclose(fp);
}

void save_tune_entry(pr_ctx *ctx, const std::vector<int64_t> &sig, int32_t mid, int32_t grid, int32_t mid_b,
                     int32_t grid_b) {
  if (ctx->tune_file.empty()) return;
  FILE *fp = fopen(ctx->tune_file.c_str(), "a");
  if (!fp) return;
  for (int64_t x : sig) fprintf(fp, "%lld ", (long long)x);
  fprintf(fp, "%d %d %d %d\n", mid, grid, mid_b, grid_b);
  fclose(fp);
}

}  // namespace prpull

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
  if (scratch_setup(device) != PR_OK) return PR_EDEVICE;
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
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hsweep, sizeof(SweepCols), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->hbstate, sizeof(BatchState), hipHostMallocDefault);
  if (e != hipSuccess) {
    set_error("pr_create: %s", hipGetErrorString(e));
    if (c->capture) (void)hipStreamDestroy(c->capture);
    if (c->hstate) (void)hipHostFree(c->hstate);
    if (c->hscratch) (void)hipHostFree(c->hscratch);
    if (c->hcols) (void)hipHostFree(c->hcols);
    if (c->hsweep) (void)hipHostFree(c->hsweep);
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
  if (ctx->hsweep) (void)hipHostFree(ctx->hsweep);
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
    // even: the updates of a chunk alternate the two row buffers from the first, so every chunk
    // must end on the buffer it started from
    if (value < 2 || value > 64 || (value & 1)) {
      set_error("batch_chunk must be even and in [2, 64]");
      return PR_EINVAL;
    }
    ctx->batch_chunk = value;
  } else if (!strcmp(key, "compact")) {
    if (value != 0 && value != 1) {
      set_error("compact must be 0 or 1");
      return PR_EINVAL;
    }
    ctx->compact = value;
  } else if (!strcmp(key, "handover32")) {
    if (value != 0 && value != 1) {
      set_error("handover32 must be 0 or 1");
      return PR_EINVAL;
    }
    ctx->handover32 = value;
  } else if (!strcmp(key, "tile") || !strcmp(key, "tile_b")) {
    // tile window of the partitions written by later prepares: entries (rows = entries / 2)
    const int part = key[4] ? 1 : 0;
    if (!valid_window(part, (int)value, (int)value / 2)) {
      set_error(part ? "tile_b must be 256 or 128" : "tile must be 1024, 512 or 256");
      return PR_EINVAL;
    }
    ctx->window_tile[part] = value;
    ctx->window_rows[part] = value / 2;
  } else if (!strcmp(key, "segmented")) {
    if (value != 0 && value != 1) {
      set_error("segmented must be 0 or 1");
      return PR_EINVAL;
    }
    ctx->segmented = value;
  } else if (!strcmp(key, "pair_mid_deg")) {
    if (value < 0 || value > kPairMax) {
      set_error("pair_mid_deg must be in [0, %d]", kPairMax);
      return PR_EINVAL;
    }
    ctx->pair_mid_deg = value;
    ctx->pair_mid_deg_set = true;
  } else if (!strcmp(key, "seg_grid")) {
    if (value < 0 || value > kMaxGrid) {
      set_error("seg_grid must be in [0, %d]", kMaxGrid);
      return PR_EINVAL;
    }
    ctx->seg_grid = value;
    ctx->seg_grid_set = value != 0;
  } else if (!strcmp(key, "seg_xcd") || !strcmp(key, "merge_xcd")) {
    if (value != 0 && value != 1) {
      set_error("%s must be 0 or 1", key);
      return PR_EINVAL;
    }
    if (key[0] == 's') {
      ctx->seg_xcd = value;
    } else {
      ctx->merge_xcd = value;
      ctx->merge_xcd_set = true;
    }
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

static bool bad_seg_args(int64_t N, int64_t E, int32_t seg_len) {
  if (bad_graph_sizes(N, E)) return true;
  if (E > 2147483646LL) {
    set_error("the source-segmented layout needs E <= 2^31-2, got %lld", (long long)E);
    return true;
  }
  if (seg_len < kMinSegLen) {
    set_error("seg_len must be at least %d, got %d", kMinSegLen, seg_len);
    return true;
  }
  return false;
}

int pr_segment_count(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, int64_t N,
                     int64_t E, int32_t seg_len, void *workspace, size_t workspace_bytes, int64_t *pairs) {
  if (!ctx || !in_offsets || !workspace || !pairs || (E > 0 && !in_indices)) {
    set_error("pr_segment_count: NULL argument");
    return PR_EINVAL;
  }
  if (bad_seg_args(N, E, seg_len)) return PR_EINVAL;
  const size_t need = (size_t)(seg_count_blocks() + 1) * sizeof(unsigned long long);
  if (workspace_bytes < need) {
    set_error("pr_segment_count: workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return PR_ENOMEM;
  }
  *pairs = 0;
  if (E == 0) return PR_OK;
  DeviceGuard g(ctx->device);
  PR_HIP(launch_seg_count((hipStream_t)stream, in_offsets, in_indices, (int32_t)N, (int32_t)E, seg_len,
                          (unsigned long long *)workspace, ctx->hscratch));
  *pairs = (int64_t)ctx->hscratch[0];
  return PR_OK;
}

size_t pr_segment_bytes(pr_ctx *ctx, int64_t N, int64_t E, int32_t seg_len, int64_t pairs) {
  if (!ctx || bad_seg_args(N, E, seg_len) || pairs < 0 || pairs > E || (E > 0 && pairs < 1)) return 0;
  if (E == 0) return prep_bytes(N, E);
  DeviceGuard g(ctx->device);
  SegLayout sl;
  if (!seg_layout(N, E, seg_len, pairs, &sl)) {
    set_error("pr_segment_bytes: hipCUB size query failed");
    return 0;
  }
  return (size_t)sl.total;
}

int pr_prepare_segmented(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, int64_t N,
                         int64_t E, int32_t seg_len, int64_t pairs, void *prep, size_t prep_bytes_) {
  if (!ctx || !in_offsets || !prep || (E > 0 && !in_indices)) {
    set_error("pr_prepare_segmented: NULL argument");
    return PR_EINVAL;
  }
  if (bad_seg_args(N, E, seg_len)) return PR_EINVAL;
  if (pairs < 0 || pairs > E || (E > 0 && pairs < 1)) {
    set_error("pr_prepare_segmented: pairs %lld out of range (use pr_segment_count)", (long long)pairs);
    return PR_EINVAL;
  }
  const size_t need = pr_segment_bytes(ctx, N, E, seg_len, pairs);
  if (need == 0) return PR_EINVAL;
  if (prep_bytes_ < need) {
    set_error("pr_prepare_segmented: prep buffer has %zu bytes, needs %zu", prep_bytes_, need);
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  int rc = prepare_into(ctx, s, in_offsets, N, E, prep, &h);
  if (rc != PR_OK || E == 0) return rc;  // no edges: the plain partitions alone
  SegLayout sl;
  if (!seg_layout(N, E, seg_len, pairs, &sl)) {
    set_error("pr_prepare_segmented: hipCUB size query failed");
    return PR_EDEVICE;
  }
  char *base = (char *)prep;
  // the count again, so that a stale or mistyped `pairs` cannot overrun the layout
  PR_HIP(launch_seg_count(s, in_offsets, in_indices, (int32_t)N, (int32_t)E, seg_len,
                          (unsigned long long *)(base + sl.cub_off), ctx->hscratch));
  if ((int64_t)ctx->hscratch[0] != pairs) {
    set_error("pr_prepare_segmented: the graph has %llu pairs at seg_len %d, %lld given", ctx->hscratch[0], seg_len,
              (long long)pairs);
    return PR_EINVAL;
  }
  PR_HIP(launch_seg_build(s, in_offsets, in_indices, (int32_t)N, (int32_t)E, seg_len, seg_key_bits(N, seg_len),
                          pairs, base, sl));
  // tile partitions of the pair CSR (P rows over E entries) and of the merge CSR (N rows over P)
  struct {
    PrepPart *pp;
    const int32_t *off;
    int64_t rows, entries;
  } parts[2] = {{&sl.pair_part, (const int32_t *)(base + sl.poff_off), pairs, E},
                {&sl.merge_part, (const int32_t *)(base + sl.moff_off), N, pairs}};
  for (auto &q : parts) {
    PrepPart &pp = *q.pp;
    PR_HIP(launch_prepare(s, pp.tile, pp.rows, q.off, q.rows, (int4 *)(base + pp.desc_off), (int4 *)(base + pp.hub_off),
                          base + sl.scan_off, ctx->hscratch));
    pp.ndesc = (int32_t)ctx->hscratch[0];
    pp.nslots = (int32_t)(ctx->hscratch[1] >> 32);
    pp.nhubs = (int32_t)(ctx->hscratch[1] & 0xffffffffull);
    if (pp.ndesc < 1 || pp.ndesc > max_desc(q.rows, q.entries, pp.tile, pp.rows) ||
        pp.nslots > max_slots(q.rows, q.entries) || pp.nhubs > max_hubs(q.rows, q.entries)) {
      set_error("internal: segmented tile partition out of bounds (ndesc %d, slots %d, hubs %d)", pp.ndesc, pp.nslots,
                pp.nhubs);
      return PR_EDEVICE;
    }
  }
  if (sl.pair_part.nhubs != 0 || sl.pair_part.nslots != 0) {
    set_error("internal: a pair longer than one tile window");
    return PR_EDEVICE;
  }
  PR_HIP(launch_seg_tile_sort(s, (int4 *)(base + sl.pair_part.desc_off), sl.pair_part.ndesc, (int32_t)E,
                              seg_key_bits(N, 1), base, sl));
  h.seg_len = seg_len;
  h.sl = sl;
  return write_prep_header(ctx, s, prep, h);
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

}  // extern "C"
