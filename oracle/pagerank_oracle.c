/*
 * pagerank_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, obviously correct CPU implementation of the standard power-iteration
 * (pull) PageRank of Sahu, Kothapalli and Banerjee, "Adjusting PageRank parameters and
 * Comparing results" (arXiv 2108.02997), in IEEE FP64.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * constant with the GPU library.
 *
 * What it computes (paper, section 2, the rank update and the common teleport
 * contribution; section 3, the three error functions; section 2, the 500-iteration cap):
 *
 *   r <- r0                                   (uniform 1/N unless a start vector is given)
 *   for k = 1 .. max_iter:
 *       D   = sum of r_u over vertices u with no out-edges
 *       c0  = (1 - alpha)/N + (alpha * D)/N
 *       for every v:  s_v = sum over v's in-edges j (ascending j) of r_{idx_j} / d_{idx_j}
 *                     r'_v = c0 + alpha * s_v
 *       e1  = sum |r'_v - r_v|,  e2 = sqrt(sum (r'_v - r_v)^2),  einf = max |r'_v - r_v|
 *       r <- r'
 *       stop when e_norm < tau  (strictly less)
 *
 * Every term comes from the previous iterate (Jacobi form).  Each contribution is a true
 * division r_u / d_u.  All sums run in ascending index order, in one thread, so results
 * are bitwise reproducible.  Only the per-vertex gather may run on several threads: every
 * r'_v is computed by one thread in the same order, so the thread count cannot change a bit.
 * Built with -O2 -ffp-contract=off and without fast-math.
 *
 * The three sums over all N vertices (D, e1 and e2^2) are compensated (Neumaier's variant of
 * Kahan summation: the rounding error of every addition is carried in a second accumulator),
 * so each is within a few units in the last place of the exact sum.  A plain running sum is
 * not: on large graphs millions of dangling vertices hold the same rank, every addition then
 * rounds the same way, and the error grows with the count (2.5e-11 relative at 2.2 million
 * terms) -- a bias of the checker, not of the method, which defines exact sums.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* Neumaier compensated summation: s + c is the running sum. */
typedef struct {
    double s, c;
} csum;

static void csum_add(csum *a, double x) {
    const double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double csum_value(const csum *a) { return a->s + a->c; }

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * norm: 1 = L1, 2 = L2, 3 = Linf.  init: N values or NULL for 1/N.  ranks: N values (out).
 * trace: max_iter x 3 values (e1, e2, einf per iteration) or NULL.  final_err: 3 values (out).
 * Returns ORC_OK when an iteration met the tolerance, ORC_NOT_CONVERGED after max_iter.
 */
int oracle_pagerank(int64_t N, const int32_t *off, const int32_t *idx, const int32_t *outdeg, double alpha,
                    double tau, int norm, int32_t max_iter, const double *init, double *ranks, double *trace,
                    int32_t *iterations, int32_t *converged, double *final_err, int nthreads) {
    if (N < 1 || !off || !outdeg || !ranks || !iterations || !converged || !final_err || max_iter < 1 ||
        norm < 1 || norm > 3 || !(alpha >= 0.0 && alpha <= 1.0) || !(tau >= 0.0))
        return ORC_EINVAL;
    if (off[N] > 0 && !idx) return ORC_EINVAL;
    double *r = (double *)malloc((size_t)N * sizeof(double));
    double *rn = (double *)malloc((size_t)N * sizeof(double));
    if (!r || !rn) {
        free(r);
        free(rn);
        return ORC_ENOMEM;
    }
    for (int64_t v = 0; v < N; ++v) r[v] = init ? init[v] : 1.0 / (double)N;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int status = ORC_NOT_CONVERGED;
    int32_t k = 0;
    double e1 = 0.0, e2 = 0.0, einf = 0.0;
    for (k = 1; k <= max_iter; ++k) {
        /* common teleport contribution, from the previous iterate */
        csum Dacc = {0.0, 0.0};
        for (int64_t u = 0; u < N; ++u)
            if (outdeg[u] == 0) csum_add(&Dacc, r[u]);
        const double D = csum_value(&Dacc);
        const double c0 = (1.0 - alpha) / (double)N + (alpha * D) / (double)N;
        /* pull: every vertex sums the contributions r_u / d_u of its in-neighbours */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1024)
#endif
        for (int64_t v = 0; v < N; ++v) {
            double s = 0.0;
            for (int64_t j = off[v]; j < off[v + 1]; ++j) {
                const int32_t u = idx[j];
                s += r[u] / (double)outdeg[u];
            }
            rn[v] = c0 + alpha * s;
        }
        /* error functions between the two successive rank vectors */
        csum sa = {0.0, 0.0}, sq = {0.0, 0.0};
        double mx = 0.0;
        for (int64_t v = 0; v < N; ++v) {
            const double d = fabs(rn[v] - r[v]);
            csum_add(&sa, d);
            csum_add(&sq, d * d);
            if (d > mx) mx = d;
        }
        e1 = csum_value(&sa);
        e2 = sqrt(csum_value(&sq));
        einf = mx;
        if (trace) {
            trace[3 * (int64_t)(k - 1) + 0] = e1;
            trace[3 * (int64_t)(k - 1) + 1] = e2;
            trace[3 * (int64_t)(k - 1) + 2] = einf;
        }
        double *t = r;
        r = rn;
        rn = t;
        const double e = norm == 1 ? e1 : (norm == 2 ? e2 : einf);
        if (e < tau) {
            status = ORC_OK;
            break;
        }
    }
    if (k > max_iter) k = max_iter;
    memcpy(ranks, r, (size_t)N * sizeof(double));
    *iterations = k;
    *converged = status == ORC_OK;
    final_err[0] = e1;
    final_err[1] = e2;
    final_err[2] = einf;
    free(r);
    free(rn);
    return status;
}
