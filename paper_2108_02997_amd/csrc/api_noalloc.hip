// api_noalloc.hip -- pr_pull_noalloc: the single solve of pr_pull for callers that cannot
// allocate device memory (serving loops, harnesses that forbid allocation).  Its workspace
// (solve state, block and hub partials, the two iterate buffers and the tile partition) lives in
// one fixed device array of this library, `scratch`, instead of a caller's buffer.
//
// In host code the name `scratch` is a host-side stand-in, not a device address: its address on
// each device is resolved once with hipGetSymbolAddress (at pr_create, with the device current)
// and only that pointer is used.  Every call on one GPU shares that GPU's array, so calls that
// overlap on one GPU (several host threads, or several streams without ordering between them)
// race; the array keeps the last call's contents, and every call rewrites what it reads (the
// solve state is cleared by a fill kernel, partials and iterates are written before they are
// read, the tile partition is rebuilt).
#include <mutex>

#include "api_internal.h"

namespace prpull {

// 64 MiB: a float64 solve of about 2 million vertices and 30 million in-edges
// (pr_workspace_bytes(N, E, precision, 1) must fit).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mutex;
static void *g_scratch_ptr[kMaxScratchDevices];

int scratch_setup(int device) {
  if (device < 0 || device >= kMaxScratchDevices) {
    set_error("device %d: the fixed scratch is kept for devices 0..%d", device, kMaxScratchDevices - 1);
    return PR_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return PR_OK;
  DeviceGuard g(device);
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    return PR_EDEVICE;
  }
  g_scratch_ptr[device] = p;
  return PR_OK;
}

static void *scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  return device >= 0 && device < kMaxScratchDevices ? g_scratch_ptr[device] : nullptr;
}

}  // namespace prpull

extern "C" {

size_t pr_noalloc_max_bytes(void) { return prpull::kScratchBytes; }

int pr_pull_noalloc(pr_ctx *ctx, void *stream, const int32_t *in_offsets, const int32_t *in_indices,
                    const int32_t *outdeg, int64_t N, int64_t E, double alpha, double tau, int32_t norm,
                    int32_t max_iter, int32_t precision, const double *init, double *ranks, double *norm_trace,
                    pr_result *out) {
  if (!ctx || !in_offsets || !outdeg || !ranks || !out || (E > 0 && !in_indices)) {
    set_error("pr_pull_noalloc: NULL argument");
    return PR_EINVAL;
  }
  if (bad_graph_sizes(N, E)) return PR_EINVAL;
  const size_t need = pr_workspace_bytes(N, E, precision, 1);
  if (need == 0) {
    set_error("pr_pull_noalloc: precision must be PR_FP64, PR_MIXED or PR_FP32, got %d", precision);
    return PR_EINVAL;
  }
  if (need > kScratchBytes) {
    set_error("pr_pull_noalloc: this graph needs %zu bytes of workspace, the fixed scratch holds %zu "
              "(N=%lld, E=%lld); use pr_pull with a workspace",
              need, kScratchBytes, (long long)N, (long long)E);
    return PR_ENOMEM;
  }
  void *ws = scratch_ptr(ctx->device);
  if (!ws) {
    set_error("pr_pull_noalloc: the fixed scratch of device %d was not resolved at pr_create", ctx->device);
    return PR_EDEVICE;
  }
  // updates launched one by one (no graph is instantiated) and not timed (no events created)
  const int64_t save_loop = ctx->loop_mode, save_timing = ctx->timing;
  ctx->loop_mode = 1;
  ctx->timing = 0;
  const int rc = pull_solve(ctx, stream, in_offsets, in_indices, outdeg, N, E, nullptr, alpha, tau, norm, max_iter,
                            precision, init, ranks, norm_trace, ws, kScratchBytes, out);
  ctx->loop_mode = save_loop;
  ctx->timing = save_timing;
  return rc;
}

}  // extern "C"
