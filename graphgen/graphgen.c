/*
 * graphgen.c -- seeded synthetic graph inputs and in-edge CSR construction.
 *
 * This module produces the inputs that both the GPU path and the CPU oracle consume.
 * It holds none of PageRank's arithmetic: it only draws edges and sorts them into the
 * in-edge compressed-row form that a pull iteration reads (for every vertex v, the
 * sources u of its in-edges, plus every vertex's out-degree d_u).
 *
 * Random numbers come from a counter-based generator: the splitmix64 finaliser
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * applied to a hash of (seed, stream, counter).  Every draw is a pure function of its
 * counter, so results do not depend on the number of threads.
 *
 * Generators:
 *   R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each edge descends `scale`
 *     levels of the adjacency matrix; at every level one uniform picks a quadrant with
 *     probabilities a, b, c, d = 1-a-b-c, as (source bit, destination bit) =
 *     (0,0), (0,1), (1,0), (1,1), most significant bit first.  No noise.  When N is not
 *     a power of two, scale = ceil(log2 N) and an edge with an endpoint >= N is redrawn
 *     (next attempt counter).
 *   Erdos-Renyi G(N, m) with a forced dangling set: the dangling set D is the first
 *     n_dangling entries of a seeded Fisher-Yates permutation; m distinct ordered pairs
 *     (u, v) with u not in D and v != u are drawn by sequential rejection of duplicates,
 *     which yields a uniform m-subset of the admissible pairs.
 *
 * CSR builder: counting sort by destination, sources sorted ascending inside each row,
 * optional removal of self-loops and of repeated (u, v) pairs; out-degrees are counted
 * from the surviving entries, so outdeg[u] always equals u's number of CSR entries.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GG_OK 0
#define GG_EINVAL (-1)
#define GG_ENOMEM (-2)

static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Counter-based draw: a pure function of (seed, stream, counter). */
uint64_t gg_hash3(uint64_t seed, uint64_t stream, uint64_t counter) {
    return mix64(mix64(mix64(seed) ^ (stream * 0xD1B54A32D192ED03ULL)) ^ counter);
}

/* Uniform double in [0,1) with 53 random bits. */
static inline double u01(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }

/* ------------------------------------------------------------------ R-MAT */

static int ceil_log2(int64_t n) {
    int s = 0;
    while (((int64_t)1 << s) < n) ++s;
    return s;
}

int gg_rmat_edges(int64_t N, int64_t m, double a, double b, double c, uint64_t seed,
                  int32_t *src, int32_t *dst, int nthreads) {
    if (N < 1 || N > 2147483647LL || m < 0 || !(a >= 0) || !(b >= 0) || !(c >= 0) ||
        a + b + c > 1.0 + 1e-12 || (m > 0 && (!src || !dst)))
        return GG_EINVAL;
    const int scale = ceil_log2(N);
    const double ab = a + b, abc = a + b + c;
    int rc = GG_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t e = 0; e < m; ++e) {
        for (uint64_t attempt = 0;; ++attempt) {
            /* one key per (edge, attempt); level l uses the l-th output of splitmix64 seeded with it */
            const uint64_t key = gg_hash3(seed, (uint64_t)e, attempt);
            uint64_t s = 0, d = 0;
            for (int l = 0; l < scale; ++l) {
                const double r = u01(mix64(key + (uint64_t)l * 0x9E3779B97F4A7C15ULL));
                const unsigned sb = r >= ab;                       /* c or d quadrant */
                const unsigned db = (r >= a && r < ab) || r >= abc; /* b or d quadrant */
                s = (s << 1) | sb;
                d = (d << 1) | db;
            }
            if ((int64_t)s < N && (int64_t)d < N) {
                src[e] = (int32_t)s;
                dst[e] = (int32_t)d;
                break;
            }
            if (attempt > 100000) { /* cannot happen for N >= 2^(scale-1) unless a == 0 etc. */
                src[e] = 0;
                dst[e] = 0;
#ifdef _OPENMP
#pragma omp atomic write
#endif
                rc = GG_EINVAL;
                break;
            }
        }
    }
    return rc;
}

/* ------------------------------------------------------------ Erdos-Renyi */

typedef struct {
    uint64_t *keys;
    uint64_t mask;
} hset;

static int hset_init(hset *h, int64_t cap_items) {
    uint64_t cap = 16;
    while (cap < (uint64_t)cap_items * 2) cap <<= 1;
    h->keys = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!h->keys) return GG_ENOMEM;
    memset(h->keys, 0xff, cap * sizeof(uint64_t)); /* empty = all ones */
    h->mask = cap - 1;
    return GG_OK;
}

/* returns 1 if inserted, 0 if present */
static int hset_insert(hset *h, uint64_t key) {
    uint64_t i = mix64(key) & h->mask;
    for (;;) {
        if (h->keys[i] == key) return 0;
        if (h->keys[i] == ~0ULL) {
            h->keys[i] = key;
            return 1;
        }
        i = (i + 1) & h->mask;
    }
}

/* Seeded permutation of [0, N) by Fisher-Yates with counter-based draws. */
int gg_permutation(int64_t N, uint64_t seed, int32_t *perm) {
    if (N < 0 || N > 2147483647LL || (N > 0 && !perm)) return GG_EINVAL;
    for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
    for (int64_t i = N - 1; i > 0; --i) {
        const uint64_t j = gg_hash3(seed, 0x5045524dULL /* "PERM" */, (uint64_t)i) % (uint64_t)(i + 1);
        const int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return GG_OK;
}

int gg_er_edges(int64_t N, int64_t m, int64_t n_dangling, uint64_t seed, int32_t *src, int32_t *dst) {
    if (N < 1 || N > 2147483647LL || m < 0 || n_dangling < 0 || n_dangling > N) return GG_EINVAL;
    const int64_t nsrc = N - n_dangling;
    /* admissible pairs: nsrc sources times (N-1) destinations */
    if ((double)m > (double)nsrc * (double)(N - 1)) return GG_EINVAL;
    if (m == 0) return GG_OK;
    if (!src || !dst) return GG_EINVAL;
    int32_t *perm = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    if (!perm) return GG_ENOMEM;
    gg_permutation(N, seed ^ 0xDA96ULL, perm);
    /* sources are perm[n_dangling .. N) */
    hset h;
    if (hset_init(&h, m) != GG_OK) {
        free(perm);
        return GG_ENOMEM;
    }
    int64_t got = 0;
    for (uint64_t k = 0; got < m; ++k) {
        const uint64_t hu = gg_hash3(seed, 0x4552554eULL, k);
        const uint64_t hv = gg_hash3(seed, 0x45525f56ULL, k);
        const int64_t u = perm[n_dangling + (int64_t)(hu % (uint64_t)nsrc)];
        int64_t v = (int64_t)(hv % (uint64_t)(N - 1));
        if (v >= u) v += 1; /* v uniform over [0,N) \ {u} */
        if (hset_insert(&h, (uint64_t)u * (uint64_t)N + (uint64_t)v)) {
            src[got] = (int32_t)u;
            dst[got] = (int32_t)v;
            ++got;
        }
    }
    free(h.keys);
    free(perm);
    return GG_OK;
}

/* --------------------------------------------------------------- CSR build */

static int cmp_i32(const void *x, const void *y) {
    const int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static void sort_row(int32_t *p, int64_t n) {
    if (n < 32) {
        for (int64_t i = 1; i < n; ++i) {
            const int32_t v = p[i];
            int64_t j = i - 1;
            while (j >= 0 && p[j] > v) {
                p[j + 1] = p[j];
                --j;
            }
            p[j + 1] = v;
        }
    } else {
        qsort(p, (size_t)n, sizeof(int32_t), cmp_i32);
    }
}

/*
 * Build the in-edge CSR of the edge list (src[e] -> dst[e]).
 * off:    N+1 entries (out); idx: capacity m entries (out, first E used); outdeg: N entries (out).
 * Returns E >= 0, or a negative status.  E must fit int32 offsets.
 */
int64_t gg_build_in_csr(int64_t N, int64_t m, const int32_t *src, const int32_t *dst, int dedupe,
                        int drop_self_loops, int32_t *off, int32_t *idx, int32_t *outdeg, int nthreads) {
    if (N < 1 || N > 2147483647LL || m < 0 || m > 2147483647LL || !off || !outdeg ||
        (m > 0 && (!src || !dst || !idx)))
        return GG_EINVAL;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t *cnt = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    if (!cnt) return GG_ENOMEM;
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] < 0 || src[e] >= N || dst[e] < 0 || dst[e] >= N) {
            free(cnt);
            return GG_EINVAL;
        }
        cnt[dst[e] + 1]++;
    }
    for (int64_t v = 0; v < N; ++v) cnt[v + 1] += cnt[v];
    int64_t *pos = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    if (!pos) {
        free(cnt);
        return GG_ENOMEM;
    }
    memcpy(pos, cnt, (size_t)N * sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) idx[pos[dst[e]]++] = src[e];
    /* per row: sort sources, then drop self-loops / repeats; new length into pos[v] */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4096)
#endif
    for (int64_t v = 0; v < N; ++v) {
        int32_t *row = idx + cnt[v];
        const int64_t n = cnt[v + 1] - cnt[v];
        sort_row(row, n);
        int64_t w = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (drop_self_loops && row[j] == (int32_t)v) continue;
            if (dedupe && w > 0 && row[w - 1] == row[j]) continue;
            row[w++] = row[j];
        }
        pos[v] = w;
    }
    /* compact in place (moves only leftwards) */
    int64_t E = 0;
    for (int64_t v = 0; v < N; ++v) {
        const int64_t n = pos[v];
        if (E != cnt[v] && n > 0) memmove(idx + E, idx + cnt[v], (size_t)n * sizeof(int32_t));
        off[v] = (int32_t)E;
        E += n;
    }
    off[N] = (int32_t)E;
    memset(outdeg, 0, (size_t)N * sizeof(int32_t));
    for (int64_t j = 0; j < E; ++j) outdeg[idx[j]]++;
    free(pos);
    free(cnt);
    return E;
}
