// relabel.h -- degree relabelling of a graph and the inverse renaming of rank vectors (relabel.hip).
#pragma once

#include "internal.h"

namespace prpull {

// Workspace bytes of launch_relabel (queries hipCUB; needs a current device).
hipError_t relabel_temp_bytes(int64_t N, int64_t E, size_t *bytes);
// host_count: pinned host word; the launch synchronises s once (to size the segmented sort).
hipError_t launch_relabel(hipStream_t s, const int32_t *off, const int32_t *idx, const int32_t *outdeg, int32_t N,
                          int32_t E, int32_t *perm, int32_t *new_off, int32_t *new_idx, int32_t *new_outdeg,
                          void *ws, size_t ws_bytes, uint32_t *host_count);
hipError_t launch_unpermute(hipStream_t s, const int32_t *perm, int32_t N, const double *in, double *out);

}  // namespace prpull
