// batch.h -- device state and parameters of the K-column solves (batch.hip).
#pragma once

#include "internal.h"

namespace prpull {

constexpr int kMaxCols = 16;

struct BatchColumn {
  double c0;        // teleport term of the column's next update
  double err[3];    // L1, L2, Linf of its last update
  double prev_l1;   // L1 of the update before (float32 stagnation test)
  int32_t iters;    // updates of this column, all phases
  int32_t fp32_iters;
  int32_t phase_updates;  // updates in the running phase (its parity names the newest buffer)
  int32_t converged;
  int32_t done;     // 1: no further updates in any phase
  int32_t active;   // 1: updated by the running phase
  int32_t met32;
  int32_t pad;
};

struct alignas(64) BatchState {
  LoopHead head;    // stop: no active column left in the running phase
  int32_t phase;    // 0: float64 solve, 1: float32 phase of a mixed solve, 2: its float64 phase
  int32_t pad[3];
  BatchColumn col[kMaxCols];
};

// Per-column parameters, in device memory (written once per solve).
struct BatchCols {
  double alpha[kMaxCols];
  double tau[kMaxCols];
  int32_t norm[kMaxCols];
  int32_t max_iter[kMaxCols];
  const double *init[kMaxCols];
  double *ranks[kMaxCols];   // NULL: k_batch_output skips the column
  double *trace[kMaxCols];
  int32_t map[kMaxCols];     // k_batch_convert / k_batch_compact: source or destination column, -1 skips
};

struct BatchParams {
  const int32_t *off;
  const int32_t *idx;
  const int32_t *outdeg;
  const int4 *desc;
  int32_t ndesc;
  int32_t N;
  const void *y_in;
  void *y_out;
  int32_t K;       // columns (problems), 1..16
  int32_t grid;    // blocks of the update launch
  int32_t nhubs;
  int32_t phase;
  int32_t mid_deg;  // rows of a tile with more entries are summed by a whole wave
  int32_t pad;
  const int4 *hubs;
  double *bpart;   // [grid][KP][4]
  double *hpart;   // [slots][KP]
  double *hacc;    // [hub blocks][KP][4]: the hub rows' error and dangling partials
  BatchState *st;
  const BatchCols *cols;
};

// Finalize column k of one update (one lane per column).
__device__ __forceinline__ void batch_finalize_column(const BatchParams &p, int k, double l1, double sq, double mx,
                                                      double dang) {
#pragma clang fp contract(off)
  BatchColumn &cs = p.st->col[k];
  const double e[3] = {l1, sqrt(sq), mx};
  cs.err[0] = e[0];
  cs.err[1] = e[1];
  cs.err[2] = e[2];
  const int32_t it = cs.iters + 1;
  cs.iters = it;
  cs.phase_updates += 1;
  if (p.phase == 1) cs.fp32_iters += 1;
  const BatchCols &cp = *p.cols;
  if (cp.trace[k]) {
    cp.trace[k][3 * (int64_t)(it - 1) + 0] = e[0];
    cp.trace[k][3 * (int64_t)(it - 1) + 1] = e[1];
    cp.trace[k][3 * (int64_t)(it - 1) + 2] = e[2];
  }
  const double N = (double)p.N;
  cs.c0 = (1.0 - cp.alpha[k]) / N + (cp.alpha[k] * dang) / N;
  const int nk = cp.norm[k];
  const bool met = (nk == 1 ? e[0] : nk == 2 ? e[1] : e[2]) < cp.tau[k];
  if (p.phase == 1) {
    if (met) cs.met32 = 1;
    if (met || !(l1 < cs.prev_l1) || (nk == 1 && l1 < kL1Handover)) cs.active = 0;
    cs.prev_l1 = l1;
    if (it >= cp.max_iter[k]) {
      cs.active = 0;
      cs.done = 1;
    }
  } else {
    if (met) {
      cs.converged = 1;
      cs.active = 0;
      cs.done = 1;
    } else if (it >= cp.max_iter[k]) {
      cs.active = 0;
      cs.done = 1;
    }
  }
}

// Hub rows (several segments) are finished kHubsPerBlock to a workgroup, one lane per (row, column).
constexpr int kHubsPerBlock = kBlock / 16;
__host__ __device__ inline int64_t hub_blocks(int64_t nhubs) { return (nhubs + kHubsPerBlock - 1) / kHubsPerBlock; }

// kp: row width, 1, 2, 4, 8, 12 or 16 values
hipError_t launch_batch_update(hipStream_t s, bool fp32, int kp, unsigned grid, const BatchParams &p);
int batch_blocks_per_cu(bool fp32, int kp);
// A float64 update whose y_in holds float32 rows (the first float64 update of a mixed batch).
hipError_t launch_batch_update_f32rows(hipStream_t s, int kp, unsigned grid, const BatchParams &p);
int batch_blocks_per_cu_f32rows(int kp);
hipError_t launch_batch_init(hipStream_t s, bool fp32, const int32_t *outdeg, int32_t N, int32_t K, int32_t kp,
                             void *y, double *bpart, int64_t bpart_blocks, const BatchParams &p, int32_t phase);
// Columns leaving the float32 phase go to a column-major float32 staging area ycol[column][N]
// (whole-line stores); launch_batch_rows then lays all K columns out as rows y[N][kp], float64
// (f64) or float32.
hipError_t launch_batch_convert(hipStream_t s, const float *y32a, const float *y32b, int32_t kp32, float *ycol,
                                int32_t N, int32_t K, const BatchState *st, const BatchCols *cols);
hipError_t launch_batch_rows(hipStream_t s, const float *ycol, void *y, bool f64, int32_t kp, int32_t N, int32_t K);
hipError_t launch_batch_rearm(hipStream_t s, BatchState *st, int32_t K);
hipError_t launch_batch_compact(hipStream_t s, bool fp32, const void *src, int32_t kp_src, void *dst, int32_t kp_dst,
                                int32_t N, int32_t K, const BatchCols *cols);
hipError_t launch_batch_output(hipStream_t s, bool fp32, const int32_t *outdeg, const void *ya, const void *yb,
                               int32_t kp, int32_t N, int32_t K, const BatchParams &p);

}  // namespace prpull
