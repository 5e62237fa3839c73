// warmstart.hip -- the learned warm start: per-vertex features from the alpha = 0.85 ranks, a
// 5 -> 32 -> 32 -> 1 ReLU perceptron (float32 weights, bfloat16 activations, float32
// accumulation), its gradient, Adam, and the start vector it proposes.  The power iteration
// (pull.hip / batch.hip) then corrects and judges the start.  Not from the paper: the paper's
// method is the iteration itself; this only chooses where it starts.
//
// Packed parameters (1281 floats): W1[32][5] | b1[32] | W2[32][32] | b2[32] | W3[32] | b3.
// Features per vertex (row of 5): log(1+indeg), log(1+outdeg), log(N r_v), log(N m_v) with m_v the
// mean of r over v's in-edges (1/N without in-edges), target alpha.
// Output y_v; proposed start r_v proportional to exp(log(N r85_v) + y_v).
#include "internal.h"
#include "device.h"

namespace prpull {

constexpr int kF = 5, kH = 32;
constexpr int oW1 = 0, oB1 = oW1 + kH * kF, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kH;
constexpr int kParams = oB3 + 1;  // 1281
constexpr int kChunk = 128;       // vertices per backward step of a block

__device__ __forceinline__ float to_bf16_float(float x) {
  // round to nearest even on the upper 16 bits (inputs are finite)
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ uint16_t bf16_bits(float x) { return (uint16_t)(__float_as_uint(x) >> 16); }
__device__ __forceinline__ float bf16_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------------ features
// The mean in-neighbour rank is a pull gather like the rank update, so it walks the same tile
// partition (prep.hip, partition A): a tile of short rows stages its index stream with coalesced
// loads and the gathered ranks in LDS, then one lane sums each row of at most kFeatLane entries
// (in entry order) and one wave each longer row; a long row that is one segment is summed by the
// block; rows of several segments (the hub table) are left to k_features_hubs, one block each.
constexpr int kFeatLane = 32;

__device__ __forceinline__ void write_features(int64_t v, int32_t deg, double s, int32_t N,
                                               const int32_t *__restrict__ outdeg, const double *__restrict__ r,
                                               double alpha_t, float *__restrict__ feat,
                                               const double *__restrict__ r_target, float *__restrict__ target) {
  const double Nd = (double)N;
  float *f = feat + v * kF;
  f[0] = (float)log1p((double)deg);
  f[1] = (float)log1p((double)outdeg[v]);
  f[2] = (float)log(Nd * r[v]);
  f[3] = deg > 0 ? (float)log(Nd * (s / (double)deg)) : 0.0f;
  f[4] = (float)alpha_t;
  if (target) target[v] = (float)log(r_target[v] / r[v]);
}

__global__ __launch_bounds__(kBlock) void k_features(const int32_t *__restrict__ off, const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ outdeg, int32_t N,
                                                     const int4 *__restrict__ desc, int32_t ndesc,
                                                     const double *__restrict__ r, double alpha_t,
                                                     float *__restrict__ feat, const double *__restrict__ r_target,
                                                     float *__restrict__ target) {
  __shared__ double vals[kSpan];
  __shared__ double red[kWaves];
  constexpr int kPer = kSpan / kBlock;
  const int t = threadIdx.x, lane = t & 63;
  for (int32_t i = blockIdx.x; i < ndesc; i += gridDim.x) {
    const int4 d = desc[i];
    const int4 dn = desc[i + 1];
    const int32_t e0 = d.y, e1 = dn.y;
    if (d.z < 0) {
      const int32_t v0 = d.x, v1 = dn.x, n = e1 - e0;
      int32_t u[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int j = t + k * kBlock;
        u[k] = j < n ? __builtin_nontemporal_load(idx + e0 + j) : -1;
      }
      int32_t ra[kRowsPerLane], rb[kRowsPerLane];
#pragma unroll
      for (int q = 0; q < kRowsPerLane; ++q) {
        const int32_t v = v0 + t + q * kBlock;
        ra[q] = rb[q] = 0;
        if (v < v1) {
          ra[q] = off[v] - e0;
          rb[q] = off[v + 1] - e0;
        }
      }
      double x[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) x[k] = u[k] >= 0 ? r[u[k]] : 0.0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int j = t + k * kBlock;
        if (j < n) vals[j] = x[k];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kRowsPerLane; ++q) {
        const int32_t v = v0 + t + q * kBlock;
        const bool mine = v < v1;
        const int32_t deg = rb[q] - ra[q];
        const bool mid = mine && deg > kFeatLane;
        double s = 0.0;
        if (mine && !mid)
          for (int32_t j = ra[q]; j < rb[q]; ++j) s += vals[j];
        unsigned long long m = __ballot(mid);
        while (m) {
          const int src = __ffsll((long long)m) - 1;
          m &= m - 1;
          const int32_t wa = __shfl(ra[q], src, 64), wb = __shfl(rb[q], src, 64);
          double w = 0.0;
          for (int32_t j = wa + lane; j < wb; j += 64) w += vals[j];
          w = wave_sum(w);
          if (lane == src) s = w;
        }
        if (mine) write_features(v, deg, s, N, outdeg, r, alpha_t, feat, r_target, target);
      }
      __syncthreads();
    } else if (d.w < 0) {
      // a long row that is a single segment [e0, e1)
      const int32_t v = d.x;
      double s = 0.0;
      for (int32_t j = e0 + t; j < e1; j += kBlock) s += r[idx[j]];
      s = block_sum(s, red);
      if (t == 0) write_features(v, e1 - e0, s, N, outdeg, r, alpha_t, feat, r_target, target);
    }
  }
}

// Rows of several segments: one block per row of the hub table.
__global__ __launch_bounds__(kBlock) void k_features_hubs(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ idx,
                                                          const int32_t *__restrict__ outdeg, const int4 *hubs,
                                                          int32_t N, const double *__restrict__ r, double alpha_t,
                                                          float *__restrict__ feat,
                                                          const double *__restrict__ r_target,
                                                          float *__restrict__ target) {
  __shared__ double red[kWaves];
  const int4 hb = hubs[blockIdx.x];
  const int32_t v = hb.x, a = off[v], b = off[v + 1];
  double s = 0.0;
  for (int32_t j = a + threadIdx.x; j < b; j += kBlock) s += r[idx[j]];
  s = block_sum(s, red);
  if (threadIdx.x == 0) write_features(v, b - a, s, N, outdeg, r, alpha_t, feat, r_target, target);
}

// ------------------------------------------------------------------ forward
__global__ __launch_bounds__(kBlock) void k_mlp_forward(const float *__restrict__ W, const float *__restrict__ feat,
                                                        int64_t N, float *__restrict__ y, uint16_t *__restrict__ act) {
  __shared__ float w[kParams];
  __shared__ float sh1[kBlock][kH + 1];  // this lane's first hidden layer
  for (int i = threadIdx.x; i < kParams; i += kBlock) w[i] = W[i];
  __syncthreads();
  float *h1 = sh1[threadIdx.x];
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock) {
    float f[kF];
#pragma unroll
    for (int i = 0; i < kF; ++i) f[i] = feat[v * kF + i];
#pragma unroll 4
    for (int j = 0; j < kH; ++j) {
      float z = w[oB1 + j];
#pragma unroll
      for (int i = 0; i < kF; ++i) z = fmaf(w[oW1 + j * kF + i], f[i], z);
      h1[j] = to_bf16_float(fmaxf(z, 0.0f));
    }
    float z2[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) z2[j] = w[oB2 + j];
#pragma unroll 1
    for (int k = 0; k < kH; ++k) {
      const float hk = h1[k];
#pragma unroll
      for (int j = 0; j < kH; ++j) z2[j] = fmaf(w[oW2 + j * kH + k], hk, z2[j]);
    }
    float out = w[oB3];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
      const float h2 = to_bf16_float(fmaxf(z2[j], 0.0f));
      out = fmaf(w[oW3 + j], h2, out);
      if (act) act[v * (2 * kH) + kH + j] = bf16_bits(h2);
    }
    y[v] = out;
    if (act) {
#pragma unroll 4
      for (int j = 0; j < kH; ++j) act[v * (2 * kH) + j] = bf16_bits(h1[j]);
    }
  }
}

// ------------------------------------------------------------------ backward (mean squared error)
// Per block: chunks of kChunk vertices; lanes < kChunk compute one vertex's dL/dz terms into LDS,
// then every lane accumulates the parameters it owns over the chunk in vertex order.  Block
// partials are reduced in block order by k_mlp_grad_reduce.
__global__ __launch_bounds__(kBlock, 2) void k_mlp_backward(const float *__restrict__ W, const float *__restrict__ feat,
                                                         const uint16_t *__restrict__ act,
                                                         const float *__restrict__ y, const float *__restrict__ target,
                                                         int64_t N, double inv_n, float *__restrict__ part,
                                                         double *__restrict__ loss_part) {
  __shared__ float w[kParams];
  __shared__ float sh1[kChunk][kH + 1], sh2[kChunk][kH + 1], sdz1[kChunk][kH + 1], sdz2[kChunk][kH + 1];
  __shared__ float sf[kChunk][kF], sdy[kChunk];
  __shared__ double red[kWaves];
  const int t = threadIdx.x;
  for (int i = t; i < kParams; i += kBlock) w[i] = W[i];
  float g2[4] = {0.f, 0.f, 0.f, 0.f};  // dW2 entries 4t .. 4t+3
  float gx = 0.f;                       // lanes 0..159 dW1, 160..191 db1, 192..223 db2, 224..255 dW3
  float gb3 = 0.f;                      // lane 0: db3
  double loss = 0.0;
  __syncthreads();
  for (int64_t base = (int64_t)blockIdx.x * kChunk; base < N; base += (int64_t)gridDim.x * kChunk) {
    if (t < kChunk) {
      const int64_t v = base + t;
      if (v < N) {
        const float d = y[v] - target[v];
        loss += (double)d * (double)d;
        const float dy = (float)(2.0 * inv_n) * d;
        sdy[t] = dy;
#pragma unroll
        for (int i = 0; i < kF; ++i) sf[t][i] = feat[v * kF + i];
#pragma unroll 4
        for (int j = 0; j < kH; ++j) {
          const float h1 = bf16_to_float(act[v * (2 * kH) + j]);
          const float h2 = bf16_to_float(act[v * (2 * kH) + kH + j]);
          sh1[t][j] = h1;
          sh2[t][j] = h2;
          sdz2[t][j] = h2 > 0.f ? dy * w[oW3 + j] : 0.f;
        }
#pragma unroll 1
        for (int k = 0; k < kH; ++k) {
          float s = 0.f;
#pragma unroll
          for (int j = 0; j < kH; ++j) s = fmaf(w[oW2 + j * kH + k], sdz2[t][j], s);
          sdz1[t][k] = sh1[t][k] > 0.f ? s : 0.f;
        }
      } else {
        sdy[t] = 0.f;
#pragma unroll
        for (int i = 0; i < kF; ++i) sf[t][i] = 0.f;
#pragma unroll
        for (int j = 0; j < kH; ++j) sh1[t][j] = sh2[t][j] = sdz1[t][j] = sdz2[t][j] = 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = 4 * t + q, j = e / kH, k = e % kH;
      float s = 0.f;
#pragma unroll 4
      for (int vv = 0; vv < kChunk; ++vv) s = fmaf(sdz2[vv][j], sh1[vv][k], s);
      g2[q] += s;
    }
    float s = 0.f;
    if (t < kH * kF) {
      const int j = t / kF, i = t % kF;
      for (int vv = 0; vv < kChunk; ++vv) s = fmaf(sdz1[vv][j], sf[vv][i], s);
    } else if (t < kH * kF + kH) {
      for (int vv = 0; vv < kChunk; ++vv) s += sdz1[vv][t - kH * kF];
    } else if (t < kH * kF + 2 * kH) {
      for (int vv = 0; vv < kChunk; ++vv) s += sdz2[vv][t - kH * kF - kH];
    } else if (t < kH * kF + 3 * kH) {
      const int j = t - kH * kF - 2 * kH;
      for (int vv = 0; vv < kChunk; ++vv) s = fmaf(sdy[vv], sh2[vv][j], s);
    }
    gx += s;
    if (t == 0) {
      float b3 = 0.f;
      for (int vv = 0; vv < kChunk; ++vv) b3 += sdy[vv];
      gb3 += b3;
    }
    __syncthreads();
  }
  float *pb = part + (int64_t)blockIdx.x * kParams;
#pragma unroll
  for (int q = 0; q < 4; ++q) pb[oW2 + 4 * t + q] = g2[q];
  if (t < kH * kF) pb[oW1 + t] = gx;
  else if (t < kH * kF + kH) pb[oB1 + t - kH * kF] = gx;
  else if (t < kH * kF + 2 * kH) pb[oB2 + t - kH * kF - kH] = gx;
  else if (t < kH * kF + 3 * kH) pb[oW3 + t - kH * kF - 2 * kH] = gx;
  if (t == 0) pb[oB3] = gb3;
  const double l = block_sum(loss, red);
  if (t == 0) loss_part[blockIdx.x] = l;
}

// Block partials [nb][kParams] -> dW.  Block x owns parameters 64x .. 64x+63; its four waves sum
// the partials of blocks b = w, w+4, w+8, ... in ascending b (float64), then the four wave sums
// are added in wave order.  Block 0 also reduces the loss partials.
constexpr int kReduceParams = 64;

__global__ __launch_bounds__(kBlock) void k_mlp_grad_reduce(const float *__restrict__ part, int32_t nb,
                                                            const double *__restrict__ loss_part, double inv_n,
                                                            float *__restrict__ dW, double *__restrict__ loss) {
  __shared__ double red[kWaves][kReduceParams];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int p = blockIdx.x * kReduceParams + lane;
  double s = 0.0;
  if (p < kParams)
    for (int32_t b = wave; b < nb; b += kWaves) s += (double)part[(int64_t)b * kParams + p];
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && p < kParams) {
    double x = red[0][lane];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) x += red[w][lane];
    dW[p] = (float)x;
  }
  if (blockIdx.x == 0) {
    __shared__ double lred[kWaves];
    double l = 0.0;
    for (int32_t b = t; b < nb; b += kBlock) l += loss_part[b];
    l = block_sum(l, lred);
    if (t == 0) *loss = l * inv_n;
  }
}

// ------------------------------------------------------------------ Adam (Kingma and Ba, Algorithm 1)
__global__ void k_adam(float *__restrict__ W, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int32_t n, float lr, float beta1, float beta2, float eps, int32_t step) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mhat = mi / (1.0f - powf(beta1, (float)step));
  const float vhat = vi / (1.0f - powf(beta2, (float)step));
  W[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

// ------------------------------------------------------------------ start vector
__global__ __launch_bounds__(kBlock) void k_start_partial(const float *__restrict__ feat, const float *__restrict__ y,
                                                          int64_t N, double *__restrict__ r0,
                                                          double *__restrict__ part) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock) {
    const double w = exp((double)feat[v * kF + 2] + (double)y[v]);
    r0[v] = w;
    s += w;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_start_scale(double *__restrict__ r0, int64_t N,
                                                        const double *__restrict__ part, int32_t nb) {
  __shared__ double red[kWaves];
  __shared__ double total;
  double s = 0.0;
  for (int32_t b = threadIdx.x; b < nb; b += kBlock) s += part[b];
  s = block_sum(s, red);
  if (threadIdx.x == 0) total = s;
  __syncthreads();
  const double inv = 1.0 / total;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < N; v += (int64_t)gridDim.x * kBlock) r0[v] *= inv;
}

// ------------------------------------------------------------------ launchers
static unsigned blocks_for(int64_t n, int64_t cap) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

int mlp_param_count() { return kParams; }
int mlp_backward_blocks(int64_t N) {
  int64_t g = (N + kChunk - 1) / kChunk;
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  return (int)g;
}

hipError_t launch_features(hipStream_t s, const int32_t *off, const int32_t *idx, const int32_t *outdeg, int32_t N,
                           const int4 *desc, int32_t ndesc, const int4 *hubs, int32_t nhubs, const double *r,
                           double alpha_t, float *feat, const double *r_target, float *target) {
  const unsigned grid = (unsigned)std::min<int64_t>(std::max<int32_t>(ndesc, 1), 4 * 2048);
  hipLaunchKernelGGL(k_features, dim3(grid), dim3(kBlock), 0, s, off, idx, outdeg, N, desc, ndesc, r, alpha_t, feat,
                     r_target, target);
  if (nhubs > 0)
    hipLaunchKernelGGL(k_features_hubs, dim3(nhubs), dim3(kBlock), 0, s, off, idx, outdeg, hubs, N, r, alpha_t, feat,
                       r_target, target);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(hipStream_t s, const float *W, const float *feat, int64_t N, float *y, uint16_t *act) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(N, 4096)), dim3(kBlock), 0, s, W, feat, N, y, act);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(hipStream_t s, const float *W, const float *feat, const uint16_t *act, const float *y,
                               const float *target, int64_t N, float *part, double *loss_part, float *dW,
                               double *loss) {
  const int nb = mlp_backward_blocks(N);
  const double inv_n = 1.0 / (double)N;
  hipLaunchKernelGGL(k_mlp_backward, dim3(nb), dim3(kBlock), 0, s, W, feat, act, y, target, N, inv_n, part,
                     loss_part);
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((kParams + kReduceParams - 1) / kReduceParams), dim3(kBlock), 0, s,
                     (const float *)part, nb,
                     (const double *)loss_part, inv_n, dW, loss);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, float *W, const float *g, float *m, float *v, int32_t n, float lr, float beta1,
                       float beta2, float eps, int32_t step) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, W, g, m, v, n, lr, beta1, beta2, eps, step);
  return hipGetLastError();
}

hipError_t launch_start_vector(hipStream_t s, const float *feat, const float *y, int64_t N, double *r0, double *part) {
  const unsigned nb = blocks_for(N, 1024);
  hipLaunchKernelGGL(k_start_partial, dim3(nb), dim3(kBlock), 0, s, feat, y, N, r0, part);
  hipLaunchKernelGGL(k_start_scale, dim3(nb), dim3(kBlock), 0, s, r0, N, (const double *)part, (int32_t)nb);
  return hipGetLastError();
}

}  // namespace prpull
