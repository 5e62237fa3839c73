/*
 * prpull.h -- C ABI of the MI355X (gfx950) pull-PageRank library, libprpull.so.
 *
 * The library computes the standard power-iteration (pull) PageRank of Sahu, Kothapalli and
 * Banerjee, "Adjusting PageRank parameters and Comparing results" (arXiv 2108.02997):
 *
 *   section 2, rank update:  r'_v = c0 + alpha * sum over v's in-edges (u -> v) of r_u / d_u,
 *                             every term taken from the previous iterate;
 *   section 2, teleport:      c0 = (1 - alpha)/N + alpha * (sum of r over dangling vertices)/N,
 *                             a dangling vertex being one with no out-edges;
 *   section 3, convergence:   stop once the L1, L2 or L-infinity norm of r' - r falls strictly
 *                             below the tolerance tau;
 *   section 2, iteration cap: at most max_iter updates (the paper uses 500), after which the
 *                             last iterate is returned as not converged.
 * The start vector is uniform 1/N unless the caller passes one (the paper does not state it).
 *
 * Conventions for every entry point
 *   - All array arguments are device pointers (memory on the context's GPU) unless marked
 *     "host".  The caller owns every buffer, including the workspace; the library allocates no
 *     device memory in pr_pull, pr_pull_batch or the warm-start calls.  A context owns only
 *     host-side caches (captured HIP graphs, pinned status words) and frees them in pr_destroy.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *     stream-ordered; calls that fill a host result synchronise the stream before returning.
 *   - Graph layout ("in-edge CSR"): in_offsets[N+1] int32, non-decreasing, in_offsets[0] = 0,
 *     in_offsets[N] = E; in_indices[E] int32, entry j of row v is the source u of an edge
 *     u -> v; outdeg[N] int32 = number of CSR entries naming u.  Repeated entries and
 *     self-loops are allowed and counted as edges.  0 <= E < 2^31.  Structure is checked only
 *     by pr_validate_graph.
 *   - Rank and trace arrays are float64.  A norm trace holds max_iter rows of (L1, L2, Linf),
 *     one row per update performed; rows past the last update are left untouched.
 *   - Return value: PR_OK (0) or PR_NOT_CONVERGED (1) when outputs are valid, a negative
 *     status when they are undefined; pr_last_error() then describes the failure (text owned
 *     by the library, valid until the next call on the same host thread).
 *   - One context per host thread; calls that overlap on one context are not supported.
 */
#ifndef PRPULL_H
#define PRPULL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pr_ctx pr_ctx;

/* Error functions of section 3. */
enum { PR_L1 = 1, PR_L2 = 2, PR_LINF = 3 };

/* Arithmetic of the solve.
 * PR_FP64:  contributions, gather, ranks, reductions all in float64.
 * PR_MIXED: a float32 phase (float32 contributions and gather with float32 accumulation;
 *           dangling sum, teleport term and norms in float64) runs until it meets tau, its L1
 *           change stops decreasing or, for the L1 norm, that change is below 2^-17; then
 *           float64 iterations continue from the float32 iterate until a float64 update meets
 *           tau.  The convergence decision is always taken on a float64 update.
 * PR_FP32:  pr_pull only, an ablation: the float32 phase alone, run until it meets tau or
 *           max_iter, with no float64 update; it shows where float32 iterates stop converging
 *           (the paper's sensitivity limits of section 4) and is not meant for results. */
enum { PR_FP64 = 0, PR_MIXED = 1, PR_FP32 = 2 };

enum {
  PR_OK = 0,
  PR_NOT_CONVERGED = 1, /* max_iter updates done without meeting tau; ranks hold the last iterate */
  PR_EINVAL = -1,       /* bad scalar argument, NULL where a buffer is required, size mismatch */
  PR_ENOMEM = -2,       /* workspace or prep buffer smaller than required */
  PR_EDEVICE = -3,      /* a HIP call failed */
  PR_EGRAPH = -4        /* pr_validate_graph found a malformed CSR */
};

typedef struct {
  int32_t iterations; /* updates performed, including the one that met tau (1..max_iter) */
  int32_t converged;  /* 1 if an update met tau (always a float64 update) */
  int32_t fp32_iters; /* updates of the float32 phase (PR_MIXED, PR_FP32), else 0 */
  int32_t fp64_iters; /* float64 updates */
  double final_err[3]; /* L1, L2, Linf of r' - r at the last update */
} pr_result;

/* ---------------------------------------------------------------- context */

/* Create a context bound to HIP device `device`.  Returns PR_OK or PR_EDEVICE. */
int pr_create(pr_ctx **out, int device);
/* Destroy a context (NULL allowed).  Waits for nothing; the caller synchronises its streams. */
void pr_destroy(pr_ctx *ctx);
/* Description of the last negative status on this host thread ("" if none). */
const char *pr_last_error(void);
/* Library version string. */
const char *pr_version(void);

/* Tunables of a context (read by later solves):
 *   "grid"  : maximum number of workgroups of an update launch, 1..16384, or 0 (default) for one
 *             workgroup per resident slot (compute units x occupancy of the update kernel)
 *   "chunk" : updates per captured HIP graph between two host checks, even, 2..64 (default 16;
 *             a host check costs tens of microseconds, an update past the stop a few)
 *   "loop"  : 0 = replay captured HIP graphs (default), 1 = launch the updates one by one
 *   "mid_deg": rows of at most this many in-edges are summed by one lane, longer rows (up to the
 *             tile window) by a whole wave64, 0..1024 (default 32); pr_pull only
 *   "tile"  : tile window of partition A written by later prepares: 1024 (default), 512 or 256
 *             entries (rows = entries / 2)
 *   "tile_b": the same for partition B (the K-column tiles): 256 (default) or 128
 *   "tuned" : 1 (default) = use the autotuner's choice for graphs it has seen (pr_autotune)
 *   "batch_chunk": updates of pr_pull_batch between two host checks, even, 2..64 (default 2)
 *   "compact": 1 (default) = when enough columns of pr_pull_batch have stopped, repack the
 *             remaining ones into narrower rows (fewer bytes per edge); 0 = keep the layout
 *   "handover32": 1 (default) = when no column of a PR_MIXED pr_pull_batch stopped at max_iter
 *             in its float32 phase, the first float64 update reads the float32 rows themselves
 *             (exact in float64, half the bytes per edge) and sums in float64; the result is
 *             bitwise the one of 0 = first lay the columns out as float64 rows
 *   "barrier_ms": time limit of one grid-barrier wait of pr_pull_multi in milliseconds, 0..600000
 *             (default 5000); a wait that passes it ends the launch with PR_EDEVICE
 *   "segmented": 1 (default) = pr_pull runs source-segmented updates when its prep buffer has the
 *             layout of pr_prepare_segmented; 0 = the plain update on the same buffer
 *   "pair_mid_deg": pairs of the per-segment step with more entries than this are summed by a
 *             whole wave64, shorter ones by one lane, 0..1024 (default 256)
 *   "seg_grid": workgroups of the per-segment step of a source-segmented update, 1..16384; 0
 *             (default) = as many as the compute units hold of the update kernel at once
 *   "seg_xcd": 1 (default) = the per-segment step of a source-segmented update gives each of the
 *             8 XCDs a contiguous eighth of its tiles (each XCD then walks a few segments of its
 *             own, and a segment's slice of the iterate is fetched into one XCD's L2 only);
 *             0 = tiles dealt round-robin over all workgroups.  Bitwise the same results
 *   "merge_xcd": 1 = the same for the merge step (neighbouring tiles read neighbouring partial
 *             sums, which then share lines in one XCD's L2: pays for short segments, with many
 *             pairs); 0 (default) = round-robin.  The ranks are bitwise the same; the norms'
 *             partial sums are grouped differently
 *   "narrow": 1 (default) = one or two columns of pr_pull_batch run on rows of one or two values;
 *             0 = rows hold at least four values (the row layouts keep every column's sums in
 *             the same order, so with a pinned grid compaction then leaves results bitwise equal)
 *   "timing": 1 = launch updates one by one, each bracketed by HIP events on the solve stream,
 *             and accumulate their durations (pr_get_stats); graphs are not replayed meanwhile
 * Returns PR_OK or PR_EINVAL for an unknown key or a value out of range. */
int pr_set_option(pr_ctx *ctx, const char *key, int64_t value);

/* Kernel kinds reported by pr_get_stats. */
enum {
  PR_KERNEL_UPDATE_F64 = 0, /* one float64 update of pr_pull */
  PR_KERNEL_UPDATE_F32 = 1, /* one float32 update (PR_MIXED first phase) */
  PR_KERNEL_BATCH_F64 = 2,  /* one float64 update of pr_pull_batch (all active columns) */
  PR_KERNEL_BATCH_F32 = 3,  /* one float32 update of pr_pull_batch */
  PR_KERNEL_MULTI = 4,      /* one whole pr_pull_multi launch (all rounds of all graphs) */
  PR_KERNEL_SWEEP_FOLD = 5, /* one fold of pr_pull_sweep (a chunk of iterates into the columns) */
  /* pr_pull_batch updates again, split by the row width (values per vertex) the update ran on:
   * widths 1, 2, 4, 8, 12, 16 are kinds ..._W1 + 0 .. 5 */
  PR_KERNEL_BATCH_F64_W1 = 8,
  PR_KERNEL_BATCH_F32_W1 = 14,
  PR_KERNEL_KINDS = 20
};

/* With "timing" on: number of timed launches of `kind` that did work (launches that found the
 * solve already stopped are not counted) and the sum of their durations in milliseconds, since
 * the context was created or pr_reset_stats was called.  Each duration spans the two events
 * around the launch. */
int pr_get_stats(pr_ctx *ctx, int32_t kind, int64_t *launches, double *milliseconds);
int pr_reset_stats(pr_ctx *ctx);

/* --------------------------------------------------------------- graph prep (once per graph) */

/* Bytes of the prep buffer for a graph with N vertices and E CSR entries (an upper bound); 0 when
 * N is outside [1, 2^31-2] or E outside [0, 2^31-1] (the int32 CSR's range, as in every call). */
size_t pr_prep_bytes(int64_t N, int64_t E);

/* Partition the rows of the in-edge CSR into work tiles by in-degree: runs of consecutive
 * low/mid in-degree rows holding about one LDS tile of entries, and high in-degree rows split
 * into fixed-size segments.  Reads only in_offsets.  Writes `prep` (device, caller-owned,
 * prep_bytes >= pr_prep_bytes(N, E)); synchronises `stream` once to read the tile count.
 * The result depends only on in_offsets and may be reused by every later solve on the graph.
 * A context remembers, by buffer address, the tile counts of the prep buffers it prepared; a buffer
 * rewritten by other means (another context, a copy) must be prepared again in this context before
 * a solve here uses it. */
int pr_prepare(pr_ctx *ctx, void *stream, const int32_t *in_offsets, int64_t N, int64_t E, void *prep,
               size_t prep_bytes);

/* Source-segmented layout, a locality preprocessing for the pull gather of section 2 (the sum of
 * each row is formed as per-segment partial sums, then their sum; the terms are the same).
 * Source ids are cut into segments of seg_len consecutive ids (seg_len >= 256), chosen so that
 * one segment's slice of the iterate (8 * seg_len bytes in float64) fits an XCD's L2.  A
 * "pair" is a run of one row's entries whose sources lie in one segment, cut every 1024 entries of
 * the row.  pr_pull, given a prep buffer written by pr_prepare_segmented (and option "segmented"
 * at its default 1), runs each update as a per-segment step over the pairs listed segment by
 * segment, writing one partial sum per pair, then a merge step that sums every row's partials
 * in segment order and applies the update's epilogue.  Within a work tile of pairs the entries
 * are gathered in source order; every pair is still summed in its own entry order.  Needs
 * E <= 2^31 - 2.
 *
 * pr_segment_count: the number of pairs of the graph at seg_len, into *pairs (host).  Reads
 * in_offsets and in_indices (device); workspace: device, >= 8200 bytes.  Synchronises the stream.
 * pr_segment_bytes: bytes of a prep buffer holding the plain tile partitions of pr_prepare and the
 * segmented layout with `pairs` pairs (construction scratch included); 0 for bad arguments.
 * pr_prepare_segmented: writes that buffer (device, caller-owned; prep_bytes >= pr_segment_bytes).
 * The pair count is taken again and must equal `pairs` (else PR_EINVAL, nothing used).  The buffer
 * serves every call that takes a prep (it contains a pr_prepare result).  It also holds the pair
 * partial sums of the solve that uses it: solves sharing one segmented prep buffer must not run
 * concurrently.  Synchronises the stream.  A graph without edges gets the plain partitions only. */
int pr_segment_count(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, int64_t N,
                     int64_t E, int32_t seg_len, void *workspace, size_t workspace_bytes, int64_t *pairs);
size_t pr_segment_bytes(pr_ctx *ctx, int64_t N, int64_t E, int32_t seg_len, int64_t pairs);
int pr_prepare_segmented(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, int64_t N,
                         int64_t E, int32_t seg_len, int64_t pairs, void *prep, size_t prep_bytes);

/* Degree ordering of the vertices, a locality preprocessing for the pull gather (the ranks of the
 * relabelled graph are those of the original, renamed): perm[v] = new id of v, vertices by
 * decreasing out-degree, ties by increasing id, so the most cited sources get consecutive ids.
 * The relabelled in-CSR goes to out_offsets[N+1], out_indices[E], out_outdeg[N]: row perm[v]
 * holds v's in-edges, each source u renamed perm[u], in ascending order.  All arrays are device
 * memory owned by the caller; the outputs must not overlap the inputs.  workspace: device,
 * pr_relabel_workspace_bytes(ctx, N, E) bytes (0 when N or E is out of range or the size query
 * fails).  Synchronises the stream once.  Solve the relabelled graph, then pr_unpermute maps its
 * ranks back. */
size_t pr_relabel_workspace_bytes(pr_ctx *ctx, int64_t N, int64_t E);
int pr_relabel(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
               int64_t N, int64_t E, int32_t *perm, int32_t *out_offsets, int32_t *out_indices, int32_t *out_outdeg,
               void *workspace, size_t workspace_bytes);

/* out[v] = in[perm[v]] for v < N (device float64 arrays, not overlapping): ranks of a graph
 * relabelled by pr_relabel, back in the original ids.  Async. */
int pr_unpermute(pr_ctx *ctx, void *stream, const int32_t *perm, int64_t N, const double *in, double *out);

/* Structural check of a CSR (debugging/tests; O(N + E)): offsets monotone with off[0] = 0 and
 * off[N] = E, every index in [0, N), and outdeg[u] equal to u's number of CSR entries.
 * Needs a device workspace of at least 4*N + 256 bytes.  Returns PR_OK or PR_EGRAPH. */
int pr_validate_graph(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                      const int32_t *outdeg, int64_t N, int64_t E, void *workspace, size_t workspace_bytes);

/* ------------------------------------------------------------------ single solve */

/* Device workspace bytes needed by pr_pull (prep == NULL adds room to prepare inside it); 0 for
 * out-of-range sizes or an unknown precision. */
size_t pr_workspace_bytes(int64_t N, int64_t E, int32_t precision, int32_t with_prep);

/* One PageRank solve (sections 2 and 3).
 *   in_offsets/in_indices/outdeg : the graph, device, N+1 / E / N entries
 *   prep      : pr_prepare output for this graph, or NULL to prepare inside the workspace
 *   alpha     : damping factor in [0, 1] (alpha = 1 is allowed: c0 = dangling sum / N)
 *   tau       : tolerance >= 0 (tau = 0 never converges; the solve then runs max_iter updates)
 *   norm      : PR_L1, PR_L2 or PR_LINF
 *   max_iter  : >= 1
 *   precision : PR_FP64, PR_MIXED or PR_FP32
 *   init      : device, N values, the start vector (any non-negative vector), or NULL for 1/N
 *   ranks     : device, N values, out: the newest iterate (may alias init)
 *   norm_trace: device, max_iter x 3 values, or NULL
 *   workspace : device, workspace_bytes >= pr_workspace_bytes(N, E, precision, prep == NULL)
 *   out       : host, filled after the stream is synchronised
 * Returns PR_OK, PR_NOT_CONVERGED, or a negative status. */
int pr_pull(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
            const int32_t *outdeg, int64_t N, int64_t E, const void *prep, double alpha, double tau,
            int32_t norm, int32_t max_iter, int32_t precision, const double *init, double *ranks,
            double *norm_trace, void *workspace, size_t workspace_bytes, pr_result *out);

/* pr_pull with rank snapshots: the tolerance study of sections 3 and 4 (the ranks at each of a
 * set of (tau, norm) stopping points) from one solve.  For each of the S pairs (snap_tau[i],
 * snap_norm[i]) the ranks at the first update whose change meets snap_tau[i] in snap_norm[i]
 * (the same test as the solve's own stop, so exactly the ranks pr_pull returns when given that
 * tau and norm and the other arguments unchanged) are written to snaps[i * N .. i * N + N) as
 * the solve runs, and that update's number to snap_iter[i].  The solve itself still stops at its
 * own (tau, norm) or max_iter: a snapshot it stops before meeting gets snap_iter[i] = 0 and its
 * row is left as it was, so give the solve the pair that is met last.
 *   S         : 1 .. 64
 *   snap_tau  : host, S values >= 0;   snap_norm: host, S values PR_L1, PR_L2 or PR_LINF
 *   snaps     : device, S x N values, out
 *   snap_iter : host, S values, out (filled when the call returns; it synchronises the stream)
 *   precision : PR_FP64 or PR_FP32 (PR_MIXED changes precision along the way: PR_EINVAL)
 * Other arguments, the workspace (pr_workspace_bytes), results and statuses as pr_pull.  An update
 * that takes snapshots adds one pass over the iterate and one N-value store per snapshot taken. */
int pr_pull_snapshots(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                      const int32_t *outdeg, int64_t N, int64_t E, const void *prep, double alpha, double tau,
                      int32_t norm, int32_t max_iter, int32_t precision, const double *init, double *ranks,
                      double *norm_trace, int32_t S, const double *snap_tau, const int32_t *snap_norm,
                      double *snaps, int32_t *snap_iter, void *workspace, size_t workspace_bytes, pr_result *out);

/* For callers that cannot allocate device memory (serving loops, code that must not call
 * hipMalloc, harnesses that forbid allocation): pr_pull with prep = NULL whose workspace is a
 * fixed device array of the library (pr_noalloc_max_bytes() = 64 MiB per GPU, resolved at
 * pr_create and held until the process ends) instead of a caller's buffer.  Same arguments,
 * results and statuses as pr_pull otherwise; the updates are launched one by one (no HIP graph
 * is instantiated) and are not timed.  Graphs whose pr_workspace_bytes(N, E, precision, 1)
 * exceeds pr_noalloc_max_bytes() (about 2 million vertices and 30 million in-edges in float64)
 * are rejected with PR_ENOMEM.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on a GPU (other host threads, or streams not ordered after each other) race. */
size_t pr_noalloc_max_bytes(void);
int pr_pull_noalloc(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                    const int32_t *outdeg, int64_t N, int64_t E, double alpha, double tau, int32_t norm,
                    int32_t max_iter, int32_t precision, const double *init, double *ranks, double *norm_trace,
                    pr_result *out);

/* ------------------------------------------------------------------ several problems, one graph */

/* One problem of a batch: the parameters of sections 2 and 3 for one rank vector. */
typedef struct {
  double alpha;     /* damping factor in [0, 1] */
  double tau;       /* tolerance >= 0 */
  int32_t norm;     /* PR_L1, PR_L2 or PR_LINF */
  int32_t max_iter; /* >= 1 */
} pr_problem;

/* Device workspace bytes of pr_pull_batch for K problems (1..16); 0 for out-of-range arguments. */
size_t pr_batch_workspace_bytes(int64_t N, int64_t E, int32_t K, int32_t precision, int32_t with_prep);

/* K problems on one graph in one pass per update over its edges: the damping-factor sweep of
 * section 2 (and any mix of tolerances and error functions of sections 3-4).  The K rank
 * vectors are iterated together as rows of a K-wide array, so each in-edge fetches one row
 * for every problem; each problem keeps its own teleport term, error, stopping decision and
 * iteration count, and stops being updated once it stops (its ranks are those of its own
 * last update, exactly as if solved alone).
 *   K          : 1..16
 *   probs      : host, K problems
 *   precision  : PR_FP64, or PR_MIXED (a float32 phase for all columns, then float64 updates
 *                until each column's float64 update meets its tau)
 *   init       : host array of K device pointers (N values each; an entry may be NULL for 1/N),
 *                or NULL for all-uniform starts
 *   ranks      : host array of K device pointers (N values each, out)
 *   norm_trace : host array of K device pointers (max_iter x 3 values each) or NULL
 *   results    : host, K entries
 * Returns PR_OK when every problem converged, PR_NOT_CONVERGED when at least one hit its
 * max_iter (see results[k].converged), or a negative status. */
int pr_pull_batch(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                  const int32_t *outdeg, int64_t N, int64_t E, const void *prep, int32_t K, const pr_problem *probs,
                  int32_t precision, const double *const *init, double *const *ranks, double *const *norm_trace,
                  void *workspace, size_t workspace_bytes, pr_result *results);

/* ------------------------------------------------------------------ the damping-factor sweep */

/* Device workspace bytes of pr_pull_sweep (0 for out-of-range sizes); with_prep as for pr_pull. */
size_t pr_sweep_workspace_bytes(int64_t N, int64_t E, int32_t with_prep);

/* K problems on one graph that differ only in damping factor, tolerance, error function and
 * max_iter, all from the uniform start: the damping-factor sweep of section 2 (with any mix of
 * the tolerances and error functions of sections 3-4), in float64, by ONE iteration.  From the
 * uniform start u, k updates of section 2's map with damping factor a give
 *     r_a(k) = a^k v_k + (1 - a) sum_{j<k} a^j v_j,   v_j = the iterates of the a = 1 map from u
 * (PageRank as a power series in the damping factor), and the change of update k, in every norm,
 * is a^k times the change of the a = 1 iteration's update k.  pr_pull_sweep runs the a = 1
 * iteration (the float64 update of pr_pull, source-segmented when prep has that layout); after
 * every update each problem's change a_k^k e_k decides its stop exactly as its own iteration
 * would (same tolerance test, same count), and every 32 updates the iterates are added with the
 * weights above into each problem's ranks.  Each result (ranks, iterations, converged, final
 * errors, trace rows) is that of problem k's own power iteration up to float64 rounding; the
 * iteration runs until the last problem stops.
 *   K          : 1..64
 *   probs      : host, K problems (any alpha in [0, 1], tau >= 0, norm, max_iter >= 1)
 *   ranks      : host array of K distinct device pointers (N float64 each, out)
 *   norm_trace : host array of K device pointers (max_iter x 3 float64 each) or NULL
 *   workspace  : device, >= pr_sweep_workspace_bytes(N, E, prep == NULL) (holds 33 iterates)
 *   results    : host, K entries (fp32_iters = 0)
 * Returns PR_OK when every problem converged, PR_NOT_CONVERGED when at least one stopped at its
 * max_iter, or a negative status. */
int pr_pull_sweep(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                  const int32_t *outdeg, int64_t N, int64_t E, const void *prep, int32_t K, const pr_problem *probs,
                  double *const *ranks, double *const *norm_trace, void *workspace, size_t workspace_bytes,
                  pr_result *results);

/* ------------------------------------------------------------------ many graphs, one launch */

/* One graph of a many-graph batch with its own parameters (sections 2 and 3). */
typedef struct {
  const int32_t *in_offsets; /* device, N+1 */
  const int32_t *in_indices; /* device, E (graph-local source ids) */
  const int32_t *outdeg;     /* device, N */
  int64_t N, E;
  const void *prep;          /* pr_prepare output of this graph, or NULL to prepare inside the workspace */
  double alpha, tau;
  int32_t norm, max_iter;
  const double *init;        /* device, N, or NULL for 1/N */
  double *ranks;             /* device, N, out */
  double *norm_trace;        /* device, max_iter x 3, or NULL */
} pr_graph_problem;

/* Device workspace bytes of pr_pull_multi for these G graphs (1..4096). */
size_t pr_multi_workspace_bytes(int32_t G, const pr_graph_problem *probs);

/* G independent problems on G graphs of any sizes, float64, in ONE persistent cooperative
 * launch: every global round updates all still-active graphs (tiles of all graphs shared among
 * all workgroups, then one workgroup per graph finishes its update); each graph stops on its own
 * rule, exactly as in pr_pull.  Graphs prepared beforehand (prep != NULL) use their tiles; the
 * tile window / lane-per-row threshold comes from the context ("mid_deg", or the autotuner).
 * probs and results are host arrays of G entries.  The rounds are separated by grid barriers
 * whose waits have a time limit (option "barrier_ms"); a wait that passes it ends the launch
 * with PR_EDEVICE.  Returns PR_OK when every graph converged, PR_NOT_CONVERGED otherwise (see
 * results[g].converged), or a negative status. */
int pr_pull_multi(pr_ctx *ctx, void *stream, int32_t G, const pr_graph_problem *probs, void *workspace,
                  size_t workspace_bytes, pr_result *results);

/* ------------------------------------------------------------------ autotuner */

typedef struct {
  int32_t mid_deg;           /* single-vector update: lane-per-row / wave-per-row threshold */
  int32_t grid;              /* single-vector update: workgroups */
  int32_t tile, rows;        /* partition A tile window (entries, rows): 1024/512, 512/256 or 256/128 */
  int32_t mid_deg_batch;     /* K-column update: group-per-row / wave-per-row threshold */
  int32_t grid_batch_factor; /* K-column update: workgroups per resident slot (1 or 2) */
  int32_t tile_batch, rows_batch; /* partition B tile window: 256/128 or 128/64 */
  int32_t candidates;        /* configurations timed */
  int32_t pad;
  double best_us;            /* mean float64 update time of the choice, microseconds */
  double default_us;         /* the same with the defaults (1024/512, threshold 32, one workgroup per slot) */
  double best_batch_us;      /* mean 8-column float32 update time of the batch choice */
  double default_batch_us;   /* the same with the defaults (256/128, threshold 32, one workgroup per slot) */
  /* source-segmented update (only when the prep buffer holds that layout; else zeros) */
  int32_t pair_mid_deg;      /* per-segment step: lane-per-pair / wave-per-pair threshold */
  int32_t seg_grid;          /* per-segment step: workgroups */
  int32_t merge_xcd;         /* merge step: 1 = each XCD a contiguous range of tiles */
  int32_t seg_candidates;    /* configurations of the segmented update timed */
  double best_seg_us;        /* mean segmented float64 update time of the choice */
  double default_seg_us;     /* the same with the defaults (256, one workgroup per slot, round-robin) */
} pr_tune_result;

/* Device workspace bytes of pr_autotune (0 for out-of-range sizes); with_prep as for pr_pull. */
size_t pr_tune_workspace_bytes(int64_t N, int64_t E, int32_t with_prep);

/* The tile windows and degree-bin thresholds of this graph's updates, chosen by timing them (the
 * hot path's partition and lane/wave/block bins, section 2 update).
 *   single-vector float64 update (pr_pull, pr_pull_multi): partition A window 1024/512, 512/256 or
 *     256/128 entries/rows (rows longer than the window are split over workgroups) x lane/wave
 *     threshold 8/16/32/64/128 x 1/2/4 workgroups per resident slot, four updates each, timed on
 *     the plain (unsegmented) update;
 *   K-column float32 update (pr_pull_batch): partition B window 256/128 or 128/64 x group/wave
 *     threshold 16/32/64 x 1/2 workgroups per resident slot, three updates of 8 columns each;
 *   when the prep buffer holds a source-segmented layout, the segmented float64 update:
 *     lane/wave threshold of the pairs 64/128/256/512 x 1/2 workgroups per resident slot for
 *     the per-segment step x merge tiles round-robin / per XCD, four updates each.
 * The chosen windows are written into the prep buffer (prep != NULL: re-partitioned in place; a
 * source-segmented layout in it is kept), and the thresholds and grids are kept in the context's
 * table, keyed by the graph's size, tile counts and windows (and segment length); pr_pull,
 * pr_pull_multi, pr_pull_batch and pr_pull_sweep then use them for graphs with that signature
 * unless the options ("grid", "mid_deg", "pair_mid_deg", "seg_grid", "merge_xcd") were set
 * explicitly or "tuned" is 0.  With the environment variable PRPULL_TUNE_FILE set, the table is
 * read at pr_create and every choice is appended to that file.  ranks: device scratch of N
 * values; workspace: device, >= pr_tune_workspace_bytes(N, E, prep == NULL).  Statistics of
 * pr_get_stats are left as they were. */
int pr_autotune(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                const int32_t *outdeg, int64_t N, int64_t E, void *prep, double *ranks, void *workspace,
                size_t workspace_bytes, pr_tune_result *out);

/* ------------------------------------------------------------------ learned warm start
 * Not in the paper (its method is the iteration; this only proposes where the iteration starts).
 * A per-vertex perceptron 5 -> 32 -> 32 -> 1 with ReLU, float32 weights, bfloat16 activations and
 * float32 accumulation.  Packed weights W (pr_mlp_param_count() = 1281 floats):
 *   W1[32][5] | b1[32] | W2[32][32] | b2[32] | W3[32] | b3
 * Features (float32 [N][5]): log(1 + in-degree), log(1 + out-degree), log(N r_v), log(N m_v) with
 * m_v the mean of r over v's in-edges (1/N without in-edges), target alpha.  The output y_v is
 * added to log(N r_v): the proposed start is r0_v proportional to exp(log(N r_v) + y_v). */
int pr_mlp_param_count(void);

/* Features from the ranks r085 (device, N float64, e.g. the alpha = 0.85 solution) into feat
 * (device, float32 [N][5]).  prep: pr_prepare output of the graph (its tile partition and hub
 * table: the mean in-neighbour rank is gathered tile by tile like an update).  For training,
 * r_target (device, N float64, the ranks at alpha_target) and target (device, N float32) may be
 * given together: target_v = log(r_target_v / r085_v), the value the network's output should take.
 * Async. */
int pr_features(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
                int64_t N, int64_t E, const void *prep, const double *r085, double alpha_target, float *feat,
                const double *r_target, float *target);

/* y = MLP(feat) (device float32 [N]); act_save (device, bfloat16 bits [N][64]: the two hidden
 * layers after ReLU, 8-byte aligned) is written for the backward pass unless NULL.  The hidden
 * layers run on the matrix cores (float32 products, float32 accumulation).  Async. */
int pr_mlp_forward(pr_ctx *ctx, void *stream, const float *W, const float *feat, int64_t N, float *y,
                   uint16_t *act_save);

/* Gradient dW (device, 1281 floats) of the mean squared error mean_v (y_v - target_v)^2 from a
 * forward pass's y and act_save (8-byte aligned); loss (host) receives the error.  Block
 * partials are reduced in a fixed order (repeatable).  workspace: device, pr_mlp_backward_workspace_bytes(N).
 * Synchronises the stream. */
size_t pr_mlp_backward_workspace_bytes(int64_t N);
int pr_mlp_backward(pr_ctx *ctx, void *stream, const float *W, const float *feat, const uint16_t *act_save,
                    const float *y, const float *target, int64_t N, float *dW, void *workspace, size_t workspace_bytes,
                    double *loss);

/* One Adam update (Kingma and Ba 2015, Algorithm 1) of W with gradient dW and moments m, v (device,
 * n_params floats each); step counts from 1.  Async. */
int pr_adam_step(pr_ctx *ctx, void *stream, float *W, const float *dW, float *m, float *v, int32_t n_params, float lr,
                 float beta1, float beta2, float eps, int32_t step);

/* The proposed start vector r0 (device, N float64, sums to 1) from feat and the MLP output y.
 * workspace: device, at least 8192 bytes.  Async. */
int pr_warm_start_vector(pr_ctx *ctx, void *stream, const float *feat, const float *y, int64_t N, double *r0,
                         void *workspace, size_t workspace_bytes);

/* L1 distance sum_v |x_v - y_v| of two device vectors of N float64 values, reduced in a fixed
 * order (section 2 reports each damping factor's ranks by this distance to the alpha = 0.85
 * ranks).  workspace: device, at least 8200 bytes.  out: host.  Synchronises the stream. */
int pr_l1_distance(pr_ctx *ctx, void *stream, const double *x, const double *y, int64_t N, void *workspace,
                   size_t workspace_bytes, double *out);

#ifdef __cplusplus
}
#endif
#endif /* PRPULL_H */
