// gather_ceiling.hip -- measurement kernels, not part of the solver: how fast can this GPU do the
// memory accesses of one pull update and nothing else?  Each kernel walks a CSR index array in
// edge order and sums y[idx[j]] (or one row of a row-major table per entry), with no row
// boundaries, LDS, barriers or epilogue.  Their times bound the update kernels from below on the
// same index array: the update cannot fetch its contributions faster than this.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kInFlight = 8;  // independent loads per lane per round

// One scalar of type T per entry.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather_scalar(const int32_t *__restrict__ idx, int64_t E,
                                                            const T *__restrict__ y, double *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kThreads * kInFlight;
  double s = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * kThreads * kInFlight + threadIdx.x; base < E; base += stride) {
    int32_t u[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) {
      const int64_t j = base + (int64_t)k * kThreads;
      u[k] = j < E ? __builtin_nontemporal_load(idx + j) : -1;
    }
    T x[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) x[k] = u[k] >= 0 ? y[u[k]] : (T)0;
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) s += (double)x[k];
  }
  out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// One row of Q float4 per entry; Q consecutive lanes fetch one row (the batch kernel's pattern).
template <int Q>
__global__ __launch_bounds__(kThreads) void k_gather_rows(const int32_t *__restrict__ idx, int64_t E,
                                                          const float4 *__restrict__ Y, double *__restrict__ out) {
  const int64_t total = E * Q;
  const int64_t stride = (int64_t)gridDim.x * kThreads * kInFlight;
  double s = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * kThreads * kInFlight + threadIdx.x; base < total; base += stride) {
    float4 x[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) {
      const int64_t g = base + (int64_t)k * kThreads;
      x[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (g < total) {
        const int32_t u = __builtin_nontemporal_load(idx + g / Q);
        x[k] = Y[(int64_t)u * Q + g % Q];
      }
    }
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) s += (double)(x[k].x + x[k].y + x[k].z + x[k].w);
  }
  out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// 48-byte rows (12 floats) fetched by 4 lanes per entry, as a 12-value row of the batch kernel
// could be: Split = true, every lane loads 3 floats (12 bytes, 4-byte aligned); Split = false,
// lanes 0..2 load one aligned float4 each and lane 3 loads nothing.
template <bool Split>
__global__ __launch_bounds__(kThreads) void k_gather_rows12(const int32_t *__restrict__ idx, int64_t E,
                                                            const float *__restrict__ Y, double *__restrict__ out) {
  const int64_t total = E * 4;
  const int64_t stride = (int64_t)gridDim.x * kThreads * kInFlight;
  double s = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * kThreads * kInFlight + threadIdx.x; base < total; base += stride) {
    float4 x[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) {
      const int64_t g = base + (int64_t)k * kThreads;
      const int q = (int)(g & 3);
      x[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (g < total) {
        const int32_t u = __builtin_nontemporal_load(idx + g / 4);
        if (Split) {
          const float *r = Y + (int64_t)u * 12 + q * 3;
          x[k] = make_float4(r[0], r[1], r[2], 0.f);
        } else if (q < 3) {
          x[k] = ((const float4 *)Y)[(int64_t)u * 3 + q];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) s += (double)(x[k].x + x[k].y + x[k].z + x[k].w);
  }
  out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// The index stream alone.
__global__ __launch_bounds__(kThreads) void k_stream(const int32_t *__restrict__ idx, int64_t E,
                                                     double *__restrict__ out) {
  int64_t s = 0;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < E; j += (int64_t)gridDim.x * kThreads)
    s += __builtin_nontemporal_load(idx + j);
  out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = (double)s;
}

}  // namespace

extern "C" {

// kind: 0 = float64 scalars, 1 = float32 scalars, 2 = index stream only, 3/4/5/6 = rows of
// 16/32/64/48 bytes (1/2/4/3 float4, one per lane); 7/8 = 48-byte rows on 4 lanes (12 bytes per
// lane / 16 bytes on 3 lanes).  idx: E device int32 entries, each in [0, N).  y: device table of N
// scalars, or N rows for the row kinds.  out: device, grid*256 doubles.  Returns the HIP error code.
int gc_run(int kind, const int32_t *idx, int64_t E, const void *y, double *out, int grid, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (grid < 1 || E < 0 || !idx || !out) return (int)hipErrorInvalidValue;
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_gather_scalar<double>, dim3(grid), dim3(kThreads), 0, s, idx, E, (const double *)y, out); break;
    case 1: hipLaunchKernelGGL(k_gather_scalar<float>, dim3(grid), dim3(kThreads), 0, s, idx, E, (const float *)y, out); break;
    case 2: hipLaunchKernelGGL(k_stream, dim3(grid), dim3(kThreads), 0, s, idx, E, out); break;
    case 3: hipLaunchKernelGGL(k_gather_rows<1>, dim3(grid), dim3(kThreads), 0, s, idx, E, (const float4 *)y, out); break;
    case 4: hipLaunchKernelGGL(k_gather_rows<2>, dim3(grid), dim3(kThreads), 0, s, idx, E, (const float4 *)y, out); break;
    case 5: hipLaunchKernelGGL(k_gather_rows<4>, dim3(grid), dim3(kThreads), 0, s, idx, E, (const float4 *)y, out); break;
    case 6: hipLaunchKernelGGL(k_gather_rows<3>, dim3(grid), dim3(kThreads), 0, s, idx, E, (const float4 *)y, out); break;
    case 7: hipLaunchKernelGGL(k_gather_rows12<true>, dim3(grid), dim3(kThreads), 0, s, idx, E, (const float *)y, out); break;
    case 8: hipLaunchKernelGGL(k_gather_rows12<false>, dim3(grid), dim3(kThreads), 0, s, idx, E, (const float *)y, out); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // extern "C"
