// sweep.hip -- the damping-factor sweep of section 2 as one power series (pr_pull_sweep).
//
// The update of section 2 is r' = a M r + (1-a)/N 1, with M r = sum over in-edges of r_u/d_u plus
// the dangling sum spread over all vertices (the teleport term c0 = (1-a)/N + a D/N).  From the
// uniform start u = 1/N, k updates give
//     r_a(k) = a^k v_k + (1-a) sum_{j<k} a^j v_j,     v_j = M^j u,
// (the expansion of PageRank in powers of the damping factor: Boldi, Santini and Vigna, "PageRank
// as a function of the damping factor", 2005), and the change of update k is
//     r_a(k) - r_a(k-1) = a^k (v_k - v_{k-1}).
// v_j are the iterates of the a = 1 update from u.  So one a = 1 iteration serves every damping
// factor: column k's change at update j is alpha_k^j times that iteration's change (in each norm),
// which decides its stop exactly as its own iteration would (finalize in pull.hip), and its ranks
// are a weighted sum of the v_j, accumulated here in chunks: the iteration keeps the iterates of
// the last chunk of updates, and k_sweep_fold adds
//     c_k(j) v_j,  c_k(j) = (1-alpha_k) alpha_k^j for j < s_k, alpha_k^s_k for j = s_k, 0 after,
// to ranks_k (s_k: the update column k stopped at, not yet known while it runs).  All weights are
// non-negative and every v_j is, so the sums lose nothing to cancellation.
#include "sweep.h"

namespace prpull {

constexpr int kFoldBlock = 256;
constexpr int kMaxFoldSlots = kSweepChunk + 1;

// The fold's weights: for every column k still collecting at updates j0 .. j0 + n - 1 (not stopped,
// or stopped at one of them), c_k(j) = (1 - alpha_k) alpha_k^j for j < s_k, alpha_k^s_k at j = s_k
// and 0 after (s_k = 0 while column k runs).  One block.
__global__ __launch_bounds__(kFoldBlock) void k_sweep_coef(const SweepCols *__restrict__ sw, int32_t K, int32_t n,
                                                           int32_t j0, FoldTable *__restrict__ ft) {
#pragma clang fp contract(off)
  __shared__ int32_t cols[kMaxSweepCols];
  __shared__ int32_t ncols;
  const int t = threadIdx.x;
  if (t == 0) {
    int32_t m = 0;
    for (int k = 0; k < K; ++k) {
      const int32_t sk = sw->stop_iter[k];
      if (sk == 0 || sk >= j0) {
        cols[m] = k;
        ft->out[m] = sw->ranks[k];
        ++m;
      }
    }
    ncols = m;
    ft->m = m;
  }
  __syncthreads();
  for (int q = t; q < ncols * n; q += kFoldBlock) {
    const int r = q / n, i = q % n;
    const int k = cols[r];
    const int32_t j = j0 + i;
    const int32_t sk = sw->stop_iter[k];
    const double a = sw->alpha[k];
    double c = 0.0;
    if (sk == 0 || j < sk)
      c = (1.0 - a) * pow(a, (double)j);
    else if (j == sk)
      c = pow(a, (double)j);
    ft->coef[r][i] = c;
  }
}

// ranks_k[x] += d_x * sum_i c_k(j0 + i) y_i[x] over the slots i < n (fused multiply-adds in
// ascending i; r_i[x] = y_i[x] d_x, d_x = 1 for a dangling x), for every column k still
// collecting at these steps; the first fold (j0 = 0, every column collecting) writes ranks_k[x] =
// that sum instead.  Eleven columns of 26 iterates are 286 multiply-adds per vertex: with
// separate multiplies and adds (and the degree applied to every iterate) the fold was bound by
// its arithmetic at 2.7 TB/s; as written it streams at about the copy rate.  The column stores
// are nontemporal (nothing reads them in this pass).
__global__ __launch_bounds__(kFoldBlock) void k_sweep_fold(const double *__restrict__ slots, int64_t stride,
                                                           int32_t first, int32_t n, int32_t j0,
                                                           const int32_t *__restrict__ outdeg, int32_t N,
                                                           const FoldTable *__restrict__ ft) {
  __shared__ double coef[kMaxSweepCols][kMaxFoldSlots];
  __shared__ double *outs[kMaxSweepCols];
  const int t = threadIdx.x;
  const int32_t m = ft->m;
  for (int q = t; q < m * kMaxFoldSlots; q += kFoldBlock) {
    const int r = q / kMaxFoldSlots, i = q % kMaxFoldSlots;
    coef[r][i] = i < n ? ft->coef[r][i] : 0.0;
  }
  for (int q = t; q < m; q += kFoldBlock) outs[q] = ft->out[q];
  __syncthreads();
  for (int64_t x = (int64_t)blockIdx.x * kFoldBlock + t; x < N; x += (int64_t)gridDim.x * kFoldBlock) {
    const int32_t dx = outdeg[x];
    const double scale = dx > 0 ? (double)dx : 1.0;
    double y[kMaxFoldSlots];
#pragma unroll
    for (int i = 0; i < kMaxFoldSlots; ++i)
      y[i] = i < n ? __builtin_nontemporal_load(slots + (int64_t)(first + i) * stride + x) : 0.0;
    for (int q = 0; q < m; ++q) {
      double *__restrict__ out = outs[q];
      double sum = 0.0;
#pragma unroll
      for (int i = 0; i < kMaxFoldSlots; ++i)
        if (i < n) sum = __builtin_fma(coef[q][i], y[i], sum);
      const double acc = j0 == 0 ? sum * scale : out[x] + sum * scale;
      __builtin_nontemporal_store(acc, &out[x]);
    }
  }
}

__global__ __launch_bounds__(kFoldBlock) void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst,
                                                         int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kFoldBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kFoldBlock)
    dst[i] = src[i];
}

static unsigned fold_grid(int64_t n) {
  int64_t g = (n + kFoldBlock - 1) / kFoldBlock;
  return (unsigned)(g < 1 ? 1 : g > 8192 ? 8192 : g);
}

hipError_t launch_sweep_fold(hipStream_t s, const double *slots, int64_t stride, int32_t first, int32_t n,
                             int32_t j0, const int32_t *outdeg, int32_t N, const SweepCols *sw, int32_t K,
                             FoldTable *ft) {
  if (n < 1 || n > kMaxFoldSlots || K < 1 || K > kMaxSweepCols) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sweep_coef, dim3(1), dim3(kFoldBlock), 0, s, sw, K, n, j0, ft);
  hipLaunchKernelGGL(k_sweep_fold, dim3(fold_grid(N)), dim3(kFoldBlock), 0, s, slots, stride, first, n, j0, outdeg,
                     N, (const FoldTable *)ft);
  return hipGetLastError();
}

hipError_t launch_copy_f64(hipStream_t s, const double *src, double *dst, int64_t n) {
  hipLaunchKernelGGL(k_copy_f64, dim3(fold_grid(n)), dim3(kFoldBlock), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace prpull
