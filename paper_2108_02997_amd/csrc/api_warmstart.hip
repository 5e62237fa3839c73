// api_warmstart.hip -- the C ABI of the learned warm start: features, the network's forward and
// backward passes, Adam and the proposed start vector.
#include <string.h>

#include "api_internal.h"

extern "C" {

int pr_mlp_param_count(void) { return mlp_param_count(); }

int pr_features(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices, const int32_t *outdeg,
                int64_t N, int64_t E, const void *prep, const double *r085, double alpha_target, float *feat,
                const double *r_target, float *target) {
  if (!ctx || !in_offsets || !outdeg || !prep || !r085 || !feat || (E > 0 && !in_indices) ||
      ((r_target == nullptr) != (target == nullptr))) {
    set_error("pr_features: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  PrepHeader h;
  const int rc = get_prep(ctx, s, prep, N, E, &h);
  if (rc != PR_OK) return rc;
  const PrepPart &part = h.part[0];
  PR_HIP(launch_features(s, in_offsets, in_indices, outdeg, (int32_t)N,
                         (const int4 *)((const char *)prep + part.desc_off), part.ndesc,
                         (const int4 *)((const char *)prep + part.hub_off), part.nhubs, r085, alpha_target, feat,
                         r_target, target));
  return PR_OK;
}

int pr_mlp_forward(pr_ctx *ctx, void *stream, const float *W, const float *feat, int64_t N, float *y,
                   uint16_t *act_save) {
  if (!ctx || !W || !feat || !y) {
    set_error("pr_mlp_forward: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1) {
    set_error("pr_mlp_forward: N must be >= 1");
    return PR_EINVAL;
  }
  if (((uintptr_t)act_save & 7) != 0) {
    set_error("pr_mlp_forward: act_save must be 8-byte aligned");
    return PR_EINVAL;
  }
  DeviceGuard g(ctx->device);
  PR_HIP(launch_mlp_forward((hipStream_t)stream, W, feat, N, y, act_save));
  return PR_OK;
}

size_t pr_mlp_backward_workspace_bytes(int64_t N) {
  if (N < 1 || N > 2147483646LL) return 0;
  const int nb = mlp_backward_blocks(N);
  return align_up(sizeof(float) * (size_t)nb * (size_t)mlp_param_count(), 256) +
         align_up(sizeof(double) * (size_t)(nb + 1), 256);
}

int pr_mlp_backward(pr_ctx *ctx, void *stream, const float *W, const float *feat, const uint16_t *act_save,
                    const float *y, const float *target, int64_t N, float *dW, void *workspace, size_t workspace_bytes,
                    double *loss) {
  if (!ctx || !W || !feat || !act_save || !y || !target || !dW || !workspace || !loss) {
    set_error("pr_mlp_backward: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1) {
    set_error("pr_mlp_backward: N must be >= 1");
    return PR_EINVAL;
  }
  if (((uintptr_t)act_save & 7) != 0) {
    set_error("pr_mlp_backward: act_save must be 8-byte aligned");
    return PR_EINVAL;
  }
  if (workspace_bytes < pr_mlp_backward_workspace_bytes(N)) {
    set_error("pr_mlp_backward: workspace has %zu bytes, needs %zu", workspace_bytes,
              pr_mlp_backward_workspace_bytes(N));
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const int nb = mlp_backward_blocks(N);
  float *part = (float *)workspace;
  double *lpart = (double *)((char *)workspace + align_up(sizeof(float) * (size_t)nb * (size_t)mlp_param_count(), 256));
  PR_HIP(launch_mlp_backward(s, W, feat, act_save, y, target, N, part, lpart, dW, lpart + nb));
  PR_HIP(hipMemcpyAsync(ctx->hscratch, lpart + nb, sizeof(double), hipMemcpyDeviceToHost, s));
  PR_HIP(hipStreamSynchronize(s));
  memcpy(loss, ctx->hscratch, sizeof(double));
  return PR_OK;
}

int pr_adam_step(pr_ctx *ctx, void *stream, float *W, const float *dW, float *m, float *v, int32_t n_params, float lr,
                 float beta1, float beta2, float eps, int32_t step) {
  if (!ctx || !W || !dW || !m || !v || n_params < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f)) {
    set_error("pr_adam_step: bad argument");
    return PR_EINVAL;
  }
  DeviceGuard g(ctx->device);
  PR_HIP(launch_adam((hipStream_t)stream, W, dW, m, v, n_params, lr, beta1, beta2, eps, step));
  return PR_OK;
}

int pr_warm_start_vector(pr_ctx *ctx, void *stream, const float *feat, const float *y, int64_t N, double *r0,
                         void *workspace, size_t workspace_bytes) {
  if (!ctx || !feat || !y || !r0 || !workspace) {
    set_error("pr_warm_start_vector: NULL argument");
    return PR_EINVAL;
  }
  if (N < 1) {
    set_error("pr_warm_start_vector: N must be >= 1");
    return PR_EINVAL;
  }
  if (workspace_bytes < 1024 * sizeof(double)) {
    set_error("pr_warm_start_vector: workspace needs 8192 bytes");
    return PR_ENOMEM;
  }
  DeviceGuard g(ctx->device);
  PR_HIP(launch_start_vector((hipStream_t)stream, feat, y, N, r0, (double *)workspace));
  return PR_OK;
}

}  // extern "C"
