// sweep.h -- the power-series sweep's fold (sweep.hip), shared with its driver (api_solve.hip).
#pragma once

#include "internal.h"

namespace prpull {

// One fold's weights (k_sweep_coef, from the columns' stop updates) for k_sweep_fold: row q is
// the q-th column still collecting at the fold's updates j0 .. j0 + n - 1.
struct FoldTable {
  double coef[kMaxSweepCols][kSweepChunk + 1];
  double *out[kMaxSweepCols];  // that column's ranks
  int32_t m;                   // columns still collecting
  int32_t pad;
};

// Fold the iterates slots[first .. first + n) (y form, steps j0 .. j0 + n - 1) of a sweep into
// every column's ranks (ft: device scratch for the fold's weights); copy one iterate slot onto
// another.
hipError_t launch_sweep_fold(hipStream_t s, const double *slots, int64_t stride, int32_t first, int32_t n,
                             int32_t j0, const int32_t *outdeg, int32_t N, const SweepCols *sw, int32_t K,
                             FoldTable *ft);
hipError_t launch_copy_f64(hipStream_t s, const double *src, double *dst, int64_t n);

}  // namespace prpull
