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
constexpr int kChunk = 128;       // vertices per block step of forward and backward (a 32-vertex tile per wave)

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

// ------------------------------------------------------------------ dense layers on MFMA
// The hidden layers are dense contractions over 32-vertex tiles, one tile per wave at a time, on
// v_mfma_f32_32x32x2f32 (float32 in, float32 accumulate).  Its operand layout (one 32x32x2
// block, lane l, h = l / 32): A[i][k] sits in lane i + 32k, B[k][j] in lane j + 32k, and item r
// of the 16 accumulators of lane l is D[row(r, h)][l % 32] with row(r, h) = 8(r/4) + 4h + r%4.
// A contraction over 32 values takes 16 steps; step s pairs the values row(s, 0) and row(s, 1),
// so a 32 x 32 result held in the accumulator layout feeds the next contraction directly: lane l
// of a "vertex column" tile holds vertex l%32 at hidden units row(r, h), which is the B operand of
// a product with that tile transposed and, for the gradients, the K-major operand over vertices.
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int mrow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Packs four bfloat16 values (already rounded) into 8 bytes, lowest unit first.
__device__ __forceinline__ uint2 pack4_bf16(float a, float b, float c, float d) {
  return make_uint2((uint32_t)bf16_bits(a) | ((uint32_t)bf16_bits(b) << 16),
                    (uint32_t)bf16_bits(c) | ((uint32_t)bf16_bits(d) << 16));
}

// ------------------------------------------------------------------ forward
// Per tile: Z1^T = [W1 | b1] [X | 1]^T (3 steps, the bias as a sixth input), H1 = bf16(relu(Z1)),
// Z2^T = W2 H1^T + b2 (16 steps), H2 = bf16(relu(Z2)), y = b3 + W3 . H2 (per lane over its 16
// units, then the two halves).  act[v] = H1[v] | H2[v] as bfloat16 when kept for training.
__global__ __launch_bounds__(kBlock) void k_mlp_forward(const float *__restrict__ W, const float *__restrict__ feat,
                                                        int64_t N, float *__restrict__ y, uint16_t *__restrict__ act) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, c = lane & 31;
  float a1[3], a2[16], b2[16], w3[16];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int f = 2 * s + h;  // input f of hidden unit c: weight, or the bias as input 5
    a1[s] = f < kF ? W[oW1 + c * kF + f] : W[oB1 + c];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    a2[r] = W[oW2 + c * kH + mrow(r, h)];  // A of step r: W2[c][row(r, h)]
    b2[r] = W[oB2 + mrow(r, h)];
    w3[r] = W[oW3 + mrow(r, h)];
  }
  const float b3 = W[oB3];
  const int64_t ntiles = (N + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles; tile += (int64_t)gridDim.x * kWaves) {
    const int64_t v = tile * 32 + c;
    const bool ok = v < N;
    floatx16 z1;
#pragma unroll
    for (int r = 0; r < 16; ++r) z1[r] = 0.f;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int f = 2 * s + h;
      const float x = ok ? (f < kF ? feat[v * kF + f] : 1.0f) : 0.f;
      z1 = mfma32(a1[s], x, z1);
    }
    // lane l: vertex c, hidden units row(r, h)
    float h1[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) h1[r] = to_bf16_float(fmaxf(z1[r], 0.f));
    floatx16 z2;
#pragma unroll
    for (int r = 0; r < 16; ++r) z2[r] = b2[r];
#pragma unroll
    for (int s = 0; s < 16; ++s) z2 = mfma32(a2[s], h1[s], z2);
    float h2[16], p = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      h2[r] = to_bf16_float(fmaxf(z2[r], 0.f));
      p = fmaf(w3[r], h2[r], p);
    }
    const float out = b3 + (p + __shfl_xor(p, 32, 64));
    if (ok) {
      if (h == 0) y[v] = out;
      if (act) {
        uint2 *row = (uint2 *)(act + v * (2 * kH));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          row[2 * q + h] = pack4_bf16(h1[4 * q], h1[4 * q + 1], h1[4 * q + 2], h1[4 * q + 3]);
          row[8 + 2 * q + h] = pack4_bf16(h2[4 * q], h2[4 * q + 1], h2[4 * q + 2], h2[4 * q + 3]);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ backward (mean squared error)
// Per tile, with dy_v = 2/n (y_v - t_v):
//   vertex columns (lane: vertex c, units row(r, h)): dZ2 = [H2 > 0] dy W3;
//   dZ1 = dZ2 W2 (16 steps) lands in unit columns (lane: unit c, vertices row(r, h)), masked by
//   [H1 > 0] loaded in the same layout, beside H2 and dy of those vertices;
//   dW2 += dZ2^T H1 and [dW1 | db1]^T += [X | 1]^T dZ1 (16 steps each, K over the tile's vertices);
//   db2, dW3 per unit lane, db3 and the loss per vertex lane.
// The four waves' sums are added in wave order into the block's partial row; k_mlp_grad_reduce
// adds the blocks in block order.
__global__ __launch_bounds__(kBlock) void k_mlp_backward(const float *__restrict__ W, const float *__restrict__ feat,
                                                         const uint16_t *__restrict__ act,
                                                         const float *__restrict__ y, const float *__restrict__ target,
                                                         int64_t N, double inv_n, float *__restrict__ part,
                                                         double *__restrict__ loss_part) {
  __shared__ float sg[kWaves][kParams];
  __shared__ double red[kWaves];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, h = lane >> 5, c = lane & 31;
  float w3v[16], bw2[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    w3v[r] = W[oW3 + mrow(r, h)];
    bw2[r] = W[oW2 + mrow(r, h) * kH + c];  // B of step r: W2[row(r, h)][c]
  }
  const float w3c = W[oW3 + c];
  const float two_n = (float)(2.0 * inv_n);
  floatx16 g2, g1;  // dW2 rows row(r, h), column c; [dW1 | db1]^T rows (inputs) row(r, h), column c
#pragma unroll
  for (int r = 0; r < 16; ++r) g2[r] = g1[r] = 0.f;
  float gb2 = 0.f, gw3 = 0.f, gb3 = 0.f;
  double loss = 0.0;
  const int64_t ntiles = (N + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles; tile += (int64_t)gridDim.x * kWaves) {
    const int64_t v0 = tile * 32, v = v0 + c;
    const bool ok = v < N;
    float dy = 0.f;
    if (ok) {
      const float d = y[v] - target[v];
      dy = two_n * d;
      if (h == 0) {
        loss += (double)d * (double)d;
        gb3 += dy;
      }
    }
    // vertex columns: dZ2 of vertex c at units row(r, h)
    float dz2v[16];
    {
      uint2 q4[4] = {make_uint2(0u, 0u), make_uint2(0u, 0u), make_uint2(0u, 0u), make_uint2(0u, 0u)};
      if (ok) {
        const uint2 *row = (const uint2 *)(act + v * (2 * kH));
#pragma unroll
        for (int q = 0; q < 4; ++q) q4[q] = row[8 + 2 * q + h];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float e[4] = {bf16_to_float((uint16_t)(q4[q].x & 0xffffu)), bf16_to_float((uint16_t)(q4[q].x >> 16)),
                            bf16_to_float((uint16_t)(q4[q].y & 0xffffu)), bf16_to_float((uint16_t)(q4[q].y >> 16))};
#pragma unroll
        for (int i = 0; i < 4; ++i) dz2v[4 * q + i] = e[i] > 0.f ? dy * w3v[4 * q + i] : 0.f;
      }
    }
    // unit columns: unit c of vertices row(r, h)
    float h1u[16], dz2u[16], xu[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t u = v0 + mrow(r, h);
      const bool uok = u < N;
      const float dyu = __shfl(dy, mrow(r, h), 64);
      const float h1 = uok ? bf16_to_float(act[u * (2 * kH) + c]) : 0.f;
      const float h2 = uok ? bf16_to_float(act[u * (2 * kH) + kH + c]) : 0.f;
      h1u[r] = h1;
      dz2u[r] = h2 > 0.f ? dyu * w3c : 0.f;
      gb2 += dz2u[r];
      gw3 = fmaf(dyu, h2, gw3);
      xu[r] = (uok && c <= kF) ? (c < kF ? feat[u * kF + c] : 1.0f) : 0.f;
    }
    floatx16 dz1;
#pragma unroll
    for (int r = 0; r < 16; ++r) dz1[r] = 0.f;
#pragma unroll
    for (int s = 0; s < 16; ++s) dz1 = mfma32(dz2v[s], bw2[s], dz1);
#pragma unroll
    for (int r = 0; r < 16; ++r) dz1[r] = h1u[r] > 0.f ? dz1[r] : 0.f;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      g2 = mfma32(dz2u[s], h1u[s], g2);
      g1 = mfma32(xu[s], dz1[s], g1);
    }
  }
  // this wave's sums into sg[wave] in packed parameter order
  float *pw = sg[wave];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j = mrow(r, h);
    pw[oW2 + j * kH + c] = g2[r];
    if (j < kF) pw[oW1 + c * kF + j] = g1[r];
    else if (j == kF) pw[oB1 + c] = g1[r];
  }
  gb2 += __shfl_xor(gb2, 32, 64);
  gw3 += __shfl_xor(gw3, 32, 64);
  if (h == 0) {
    pw[oB2 + c] = gb2;
    pw[oW3 + c] = gw3;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) gb3 += __shfl_xor(gb3, o, 64);
  if (lane == 0) pw[oB3] = gb3;
  __syncthreads();
  float *pb = part + (int64_t)blockIdx.x * kParams;
  for (int i = t; i < kParams; i += kBlock) {
    float x = sg[0][i];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) x += sg[w][i];
    pb[i] = x;
  }
  const double l = block_sum(loss, red);
  if (t == 0) loss_part[blockIdx.x] = l;
}

// Block partials [nb][kParams] -> dW.  Block x owns parameters 64x .. 64x+63; its sixteen waves
// sum the partials of blocks b = w, w+16, w+32, ... in ascending b (float64), then the sixteen
// wave sums are added in wave order.  Block 0 also reduces the loss partials.
constexpr int kReduceParams = 64;
constexpr int kReduceWaves = 16;

__global__ __launch_bounds__(64 * kReduceWaves) void k_mlp_grad_reduce(const float *__restrict__ part, int32_t nb,
                                                                       const double *__restrict__ loss_part,
                                                                       double inv_n, float *__restrict__ dW,
                                                                       double *__restrict__ loss) {
  __shared__ double red[kReduceWaves][kReduceParams];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int p = blockIdx.x * kReduceParams + lane;
  double s = 0.0;
  if (p < kParams)
    for (int32_t b = wave; b < nb; b += kReduceWaves) s += (double)part[(int64_t)b * kParams + p];
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && p < kParams) {
    double x = red[0][lane];
#pragma unroll
    for (int w = 1; w < kReduceWaves; ++w) x += red[w][lane];
    dW[p] = (float)x;
  }
  if (blockIdx.x == 0) {
    __shared__ double lred[kReduceWaves];
    double l = 0.0;
    for (int32_t b = t; b < nb; b += 64 * kReduceWaves) l += loss_part[b];
    l = block_sum_n<64 * kReduceWaves>(l, lred);
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
  int64_t g = (N + kChunk - 1) / kChunk;
  g = g < 1 ? 1 : g > 4096 ? 4096 : g;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)g), dim3(kBlock), 0, s, W, feat, N, y, act);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(hipStream_t s, const float *W, const float *feat, const uint16_t *act, const float *y,
                               const float *target, int64_t N, float *part, double *loss_part, float *dW,
                               double *loss) {
  const int nb = mlp_backward_blocks(N);
  const double inv_n = 1.0 / (double)N;
  hipLaunchKernelGGL(k_mlp_backward, dim3(nb), dim3(kBlock), 0, s, W, feat, act, y, target, N, inv_n, part,
                     loss_part);
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((kParams + kReduceParams - 1) / kReduceParams), dim3(64 * kReduceWaves), 0, s,
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
