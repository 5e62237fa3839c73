/* Host-code check run under AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py (CPU only, no GPU needed).
 *
 * Part 1 (built without WITH_PRPULL, with gcc): the seeded graph generator and the CPU oracle on small graphs -- R-MAT and
 * Erdos-Renyi edge draws, in-edge CSR builds with and without deduplication, oracle solves in
 * every norm with and without a trace and a start vector, and their argument checks.
 * Part 2 (built with -DWITH_PRPULL and linked to a libprpull.so whose host code is
 * instrumented): the C-ABI entry points of
 * libprpull.so on their host-side argument paths -- NULL pointers, out-of-range sizes and
 * parameters, size queries -- which must return their documented status without touching a
 * device.  Exit status 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int gg_rmat_edges(int64_t N, int64_t m, double a, double b, double c, uint64_t seed, int32_t *src, int32_t *dst,
                  int nthreads);
int gg_er_edges(int64_t N, int64_t m, int64_t n_dangling, uint64_t seed, int32_t *src, int32_t *dst);
int gg_permutation(int64_t N, uint64_t seed, int32_t *perm);
int64_t gg_build_in_csr(int64_t N, int64_t m, const int32_t *src, const int32_t *dst, int dedupe,
                        int drop_self_loops, int32_t *off, int32_t *idx, int32_t *outdeg, int nthreads);
int oracle_pagerank(int64_t N, const int32_t *off, const int32_t *idx, const int32_t *outdeg, double alpha,
                    double tau, int norm, int32_t max_iter, const double *init, double *ranks, double *trace,
                    int32_t *iterations, int32_t *converged, double *final_err, int nthreads);

static int failures = 0;
#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);    \
      ++failures;                                                            \
    }                                                                        \
  } while (0)

static void solve_all_norms(int64_t N, const int32_t *off, const int32_t *idx, const int32_t *outdeg) {
  double *ranks = malloc(sizeof(double) * (size_t)N);
  double *init = malloc(sizeof(double) * (size_t)N);
  double *trace = malloc(sizeof(double) * 3 * 64);
  for (int64_t v = 0; v < N; ++v) init[v] = (v % 3 == 0) ? 3.0 / (double)N : 0.0;
  for (int norm = 1; norm <= 3; ++norm) {
    for (int threads = 1; threads <= 2; ++threads) {
      int32_t it = 0, conv = 0;
      double err[3];
      const int rc = oracle_pagerank(N, off, idx, outdeg, 0.85, 1e-9, norm, 64, threads == 1 ? NULL : init, ranks,
                                     trace, &it, &conv, err, threads);
      CHECK(rc >= 0 && it >= 1 && it <= 64);
      double s = 0.0;
      for (int64_t v = 0; v < N; ++v) s += ranks[v];
      CHECK(fabs(s - 1.0) < 1e-9);
    }
  }
  int32_t it = 0, conv = 0;
  double err[3];
  CHECK(oracle_pagerank(N, off, idx, outdeg, 1.5, 1e-9, 1, 8, NULL, ranks, NULL, &it, &conv, err, 1) < 0);
  CHECK(oracle_pagerank(N, off, idx, outdeg, 0.85, 1e-9, 4, 8, NULL, ranks, NULL, &it, &conv, err, 1) < 0);
  CHECK(oracle_pagerank(N, off, idx, outdeg, 0.85, 1e-9, 1, 0, NULL, ranks, NULL, &it, &conv, err, 1) < 0);
  CHECK(oracle_pagerank(N, off, idx, outdeg, 0.85, NAN, 1, 8, NULL, ranks, NULL, &it, &conv, err, 1) < 0);
  free(ranks);
  free(init);
  free(trace);
}

static void generator_and_oracle(void) {
  const int64_t N = 3000, m = 30000;
  int32_t *src = malloc(sizeof(int32_t) * (size_t)m), *dst = malloc(sizeof(int32_t) * (size_t)m);
  int32_t *off = malloc(sizeof(int32_t) * (size_t)(N + 1)), *idx = malloc(sizeof(int32_t) * (size_t)m);
  int32_t *outdeg = malloc(sizeof(int32_t) * (size_t)N), *perm = malloc(sizeof(int32_t) * (size_t)N);
  /* R-MAT on a non-power-of-two vertex count (edges with an endpoint >= N are drawn again) */
  CHECK(gg_rmat_edges(N, m, 0.57, 0.19, 0.19, 7, src, dst, 2) == 0);
  for (int dedupe = 0; dedupe <= 1; ++dedupe) {
    const int64_t E = gg_build_in_csr(N, m, src, dst, dedupe, dedupe, off, idx, outdeg, 2);
    CHECK(E > 0 && E <= m && off[N] == E);
    if (E > 0) solve_all_norms(N, off, idx, outdeg);
  }
  /* Erdos-Renyi with a forced dangling set */
  CHECK(gg_er_edges(N, 8 * N / 2, N / 20, 1, src, dst) == 0);
  const int64_t E = gg_build_in_csr(N, 8 * N / 2, src, dst, 1, 1, off, idx, outdeg, 1);
  CHECK(E > 0);
  if (E > 0) solve_all_norms(N, off, idx, outdeg);
  CHECK(gg_permutation(N, 5, perm) == 0);
  /* argument checks */
  CHECK(gg_rmat_edges(0, m, 0.57, 0.19, 0.19, 7, src, dst, 1) < 0);
  CHECK(gg_build_in_csr(N, m, src, dst, 1, 1, NULL, idx, outdeg, 1) < 0);
  src[0] = (int32_t)N; /* out of range: rejected, nothing written past the arrays */
  CHECK(gg_build_in_csr(N, m, src, dst, 1, 1, off, idx, outdeg, 1) < 0);
  free(src);
  free(dst);
  free(off);
  free(idx);
  free(outdeg);
  free(perm);
}

#ifdef WITH_PRPULL
#include "../../include/prpull.h"

static void abi_argument_paths(void) {
  CHECK(pr_version() != NULL && strlen(pr_version()) > 0);
  CHECK(pr_prep_bytes(0, 10) == 0);
  CHECK(pr_prep_bytes(10, -1) == 0);
  CHECK(pr_prep_bytes(1000, 5000) > 0);
  CHECK(pr_workspace_bytes(1000, 5000, 7, 1) == 0);
  CHECK(pr_workspace_bytes(1000, 5000, PR_FP64, 1) > pr_workspace_bytes(1000, 5000, PR_FP64, 0));
  CHECK(pr_batch_workspace_bytes(1000, 5000, 0, PR_FP64, 1) == 0);
  CHECK(pr_batch_workspace_bytes(1000, 5000, 17, PR_MIXED, 1) == 0);
  CHECK(pr_batch_workspace_bytes(1000, 5000, 11, PR_MIXED, 1) > 0);
  CHECK(pr_multi_workspace_bytes(0, NULL) == 0);
  CHECK(pr_mlp_param_count() == 1281);
  pr_ctx *ctx = NULL;
  CHECK(pr_create(NULL, 0) == PR_EINVAL);
  CHECK(pr_create(&ctx, -1) < 0 && ctx == NULL);
  CHECK(pr_last_error() != NULL);
  pr_destroy(NULL);
  pr_result res;
  CHECK(pr_pull(NULL, NULL, NULL, NULL, NULL, 10, 10, NULL, 0.85, 1e-6, PR_L1, 10, PR_FP64, NULL, NULL, NULL, NULL, 0,
                &res) == PR_EINVAL);
  CHECK(strlen(pr_last_error()) > 0);
  CHECK(pr_pull_batch(NULL, NULL, NULL, NULL, NULL, 10, 10, NULL, 2, NULL, PR_FP64, NULL, NULL, NULL, NULL, 0,
                      NULL) == PR_EINVAL);
  CHECK(pr_pull_multi(NULL, NULL, 1, NULL, NULL, 0, NULL) == PR_EINVAL);
  CHECK(pr_set_option(NULL, "chunk", 4) == PR_EINVAL);
  CHECK(pr_get_stats(NULL, 0, NULL, NULL) == PR_EINVAL);
  CHECK(pr_prepare(NULL, NULL, NULL, 10, 10, NULL, 0) == PR_EINVAL);
  CHECK(pr_validate_graph(NULL, NULL, NULL, NULL, NULL, 10, 10, NULL, 0) == PR_EINVAL);
  CHECK(pr_unpermute(NULL, NULL, NULL, 10, NULL, NULL) == PR_EINVAL);
  CHECK(pr_features(NULL, NULL, NULL, NULL, NULL, 10, 10, NULL, NULL, 0.9, NULL, NULL, NULL) == PR_EINVAL);
  CHECK(pr_mlp_forward(NULL, NULL, NULL, NULL, 10, NULL, NULL) == PR_EINVAL);
  CHECK(pr_adam_step(NULL, NULL, NULL, NULL, NULL, NULL, 10, 1e-3f, 0.9f, 0.999f, 1e-8f, 1) == PR_EINVAL);
  CHECK(pr_l1_distance(NULL, NULL, NULL, NULL, 10, NULL, 0, NULL) == PR_EINVAL);
}
#endif

int main(void) {
#ifdef WITH_PRPULL
  abi_argument_paths();
#else
  generator_and_oracle();
#endif
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("host paths ok\n");
  return 0;
}
