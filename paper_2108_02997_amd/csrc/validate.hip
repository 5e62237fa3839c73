// validate.hip -- structural check of an in-edge CSR (debugging and tests).
#include "internal.h"

namespace prpull {

// flags[0]: offsets broken, flags[1]: index out of range, flags[2]: out-degree mismatch;
// flags[3..5]: the smallest offending position of each kind (or INT_MAX).
__global__ void k_check_offsets(const int32_t *__restrict__ off, int32_t N, int32_t E, int32_t *flags) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= N; v += (int64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    if (v == 0) bad = off[0] != 0;
    else bad = off[v] < off[v - 1];
    if (v == N) bad = bad || off[N] != E;
    if (bad) {
      atomicOr(&flags[0], 1);
      atomicMin(&flags[3], (int32_t)v);
    }
  }
}

__global__ void k_count_sources(const int32_t *__restrict__ idx, int32_t N, int32_t E, uint32_t *cnt, int32_t *flags) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < E; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = idx[j];
    if (u < 0 || u >= N) {
      atomicOr(&flags[1], 1);
      atomicMin(&flags[4], (int32_t)j);
    } else {
      atomicAdd(&cnt[u], 1u);
    }
  }
}

__global__ void k_check_degrees(const int32_t *__restrict__ outdeg, const uint32_t *__restrict__ cnt, int32_t N,
                                int32_t *flags) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (int64_t)gridDim.x * blockDim.x) {
    if ((uint32_t)outdeg[v] != cnt[v] || outdeg[v] < 0) {
      atomicOr(&flags[2], 1);
      atomicMin(&flags[5], (int32_t)v);
    }
  }
}

hipError_t launch_validate(hipStream_t s, const int32_t *off, const int32_t *idx, const int32_t *outdeg, int32_t N,
                           int32_t E, uint32_t *cnt, int32_t *flags, int32_t *host_flags) {
  hipError_t e = launch_fill_u32(s, cnt, N, 0u);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(s, (uint32_t *)flags, 3, 0u);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(s, (uint32_t *)flags + 3, 3, 0x7fffffffu);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_offsets, dim3(1024), dim3(256), 0, s, off, N, E, flags);
  if (E > 0 && idx) {
    // a broken offset array does not stop the index checks: they only read idx[0..E)
    hipLaunchKernelGGL(k_count_sources, dim3(2048), dim3(256), 0, s, idx, N, E, cnt, flags);
  }
  hipLaunchKernelGGL(k_check_degrees, dim3(1024), dim3(256), 0, s, outdeg, cnt, N, flags);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host_flags, flags, 6 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace prpull
