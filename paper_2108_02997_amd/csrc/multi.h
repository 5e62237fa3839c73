// multi.h -- device structures of the many-graph persistent solve (multi.hip).
#pragma once

#include "device.h"

namespace prpull {

struct MultiGraph {
  const int32_t *off;
  const int32_t *idx;
  const int32_t *outdeg;
  const int4 *desc;    // partition A tiles of this graph (sentinel included)
  const int4 *hubs;
  double *hpart;       // hub segment partial sums
  double *y[2];        // iterate buffers
  const double *init;  // start vector or null (1/N)
  double *ranks;       // output
  double *trace;       // [max_iter][3] or null
  double alpha;
  double tau;
  int32_t N;
  int32_t nhubs;
  int32_t norm;
  int32_t max_iter;
  int32_t mid_deg;
  int32_t pslot;       // first of its min(tiles, grid) update partial slots in MultiParams::part
};

struct MultiGraphState {
  double c0;
  double err[3];
  int32_t iters;
  int32_t active;
  int32_t converged;
  int32_t pad;
};

// Grid barrier state of the cooperative launch (zeroed before it).  Counters only grow; the
// words are 128 bytes apart.  XCC_ID, the workgroup's XCD, is a 4-bit hardware field.
constexpr int kMaxXcd = 16;
constexpr int kBarPad = 32;
struct GridBarrier {
  uint32_t members[kMaxXcd * kBarPad];  // workgroups of the launch on each XCD
  uint32_t xcd[kMaxXcd * kBarPad];      // arrivals on each XCD, all barriers so far
  uint32_t release[kMaxXcd * kBarPad];  // per XCD: the last barrier its workgroups may leave
  uint32_t global[kBarPad];             // XCD arrivals, all barriers so far
  uint32_t timeout[kBarPad];            // nonzero: a wait passed its time limit (all workgroups quit)
};

struct MultiParams {
  const MultiGraph *graphs;
  MultiGraphState *states;
  const int32_t *tile_base;  // [G+1]: first global tile of each graph
  double *part;              // [slots][4]: graph g's update partials from slot graphs[g].pslot on
  double *init_part;         // [G][init blocks]: dangling sums of the start vectors
  GridBarrier *bar;
  uint64_t wait_ticks;       // time limit of a barrier wait, in wall-clock ticks
  int32_t G;
  int32_t total_tiles;
  int32_t max_rounds;
  int32_t pad;
};

int multi_blocks_per_cu();
hipError_t launch_multi(hipStream_t s, unsigned grid, const MultiParams &p, int32_t init_blocks);

}  // namespace prpull
