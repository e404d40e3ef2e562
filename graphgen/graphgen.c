/*
 * graphgen.c -- seeded synthetic graph generators (input preparation only).
 *
 * This module builds the undirected simple graphs that every test, the
 * benchmark and the oracle consume.  It holds none of the k-clique method's
 * arithmetic: it only draws random edges and writes a clean CSR (rows sorted
 * ascending, symmetric, no self-loops, no duplicate entries), which is the
 * input model of the paper's problem statement (Section 2: unweighted,
 * undirected simple graph; Section 6.1: directions, weights and self-loops are
 * dropped before any algorithm runs).
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), one stream per generator call.
 *
 * Generators:
 *   gg_er        Erdos-Renyi G(n,p) by geometric skipping over the pairs i>j
 *                (Batagelj and Brandes, "Efficient generation of large random
 *                networks", Phys. Rev. E 71, 2005).
 *   gg_rmat      R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): each sample
 *                picks one of four quadrants at every one of `scale` levels.
 *   gg_chung_lu  Chung-Lu expected-degree graph with a shifted power law of
 *                weights, sampled with the Miller-Hagberg skipping method
 *                ("Efficient generation of networks with given expected
 *                degrees", WAW 2011).
 *   gg_plant     adds cliques on uniformly drawn vertex sets (Floyd sampling).
 *   gg_from_edges builds a clean CSR from an arbitrary edge list.
 *
 * Every function returns 0 on success and a negative value on allocation
 * failure or bad arguments.  Output CSR arrays are malloc'd and owned by the
 * caller, who releases them with gg_free.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n;
    int64_t nnz;      /* = 2m directed entries */
    int32_t *row_ptr; /* n+1 entries; int32 is enough for nnz < 2^31 */
    int32_t *col_idx; /* nnz entries */
} gg_csr;

/* ---------------------------------------------------------------- RNG */
typedef struct { uint64_t s; } gg_rng;

static inline uint64_t sm64_next(gg_rng *r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* uniform double in [0,1) with 53 random bits */
static inline double sm64_unif(gg_rng *r) { return (double)(sm64_next(r) >> 11) * 0x1.0p-53; }
/* uniform integer in [0, bound) by rejection (no modulo bias) */
static inline uint64_t sm64_below(gg_rng *r, uint64_t bound) {
    uint64_t lim = UINT64_MAX - (UINT64_MAX % bound);
    uint64_t x;
    do { x = sm64_next(r); } while (x >= lim);
    return x % bound;
}

uint64_t gg_splitmix64(uint64_t x) { gg_rng r = {x}; return sm64_next(&r); }

/* ------------------------------------------------------- edge buffers */
typedef struct { uint64_t *k; int64_t n, cap; } ebuf;

static int eb_push(ebuf *b, uint32_t u, uint32_t v) {
    if (u == v) return 0; /* self-loops are dropped */
    if (b->n == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1 << 16;
        uint64_t *nk = (uint64_t *)realloc(b->k, (size_t)nc * sizeof(uint64_t));
        if (!nk) return -1;
        b->k = nk; b->cap = nc;
    }
    uint32_t a = u < v ? u : v, c = u < v ? v : u;
    b->k[b->n++] = ((uint64_t)a << 32) | c;
    return 0;
}

/* LSD radix sort of 64-bit keys, 16 bits per pass. */
static int radix_sort_u64(uint64_t *a, int64_t n) {
    if (n < 2) return 0;
    uint64_t *tmp = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    int64_t *cnt = (int64_t *)malloc(65536 * sizeof(int64_t));
    if (!tmp || !cnt) { free(tmp); free(cnt); return -1; }
    uint64_t *src = a, *dst = tmp;
    for (int pass = 0; pass < 4; ++pass) {
        int sh = pass * 16;
        memset(cnt, 0, 65536 * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) cnt[(src[i] >> sh) & 0xFFFF]++;
        int64_t s = 0;
        for (int d = 0; d < 65536; ++d) { int64_t c = cnt[d]; cnt[d] = s; s += c; }
        for (int64_t i = 0; i < n; ++i) dst[cnt[(src[i] >> sh) & 0xFFFF]++] = src[i];
        uint64_t *t = src; src = dst; dst = t;
    }
    /* after 4 passes the data is back in `a` */
    free(tmp); free(cnt);
    return 0;
}

/* Sort + dedupe the (min,max) keys and write a symmetric CSR with sorted rows. */
static int eb_to_csr(ebuf *b, int32_t n, gg_csr *out) {
    if (radix_sort_u64(b->k, b->n)) return -1;
    int64_t m = 0;
    for (int64_t i = 0; i < b->n; ++i)
        if (i == 0 || b->k[i] != b->k[i - 1]) b->k[m++] = b->k[i];
    if (2 * m > INT32_MAX) return -2;
    int32_t *rp = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *ci = (int32_t *)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int32_t));
    int32_t *fill = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!rp || !ci || !fill) { free(rp); free(ci); free(fill); return -1; }
    for (int64_t i = 0; i < m; ++i) {
        rp[(b->k[i] >> 32) + 1]++;
        rp[(uint32_t)b->k[i] + 1]++;
    }
    for (int32_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    memcpy(fill, rp, (size_t)n * sizeof(int32_t));
    /* Keys are sorted by (a,c) with a<c.  Row x receives its smaller
     * neighbours (as the `c` side of keys (w,x), w ascending) before its
     * larger ones (as the `a` side of keys (x,w), w ascending); emitting the
     * two kinds in one ascending sweep over keys would interleave them, so do
     * two sweeps: first all "lower" entries, then all "upper" entries. */
    for (int64_t i = 0; i < m; ++i) { /* entry (c -> a): a < c, a ascending per row c */
        uint32_t a = (uint32_t)(b->k[i] >> 32), c = (uint32_t)b->k[i];
        ci[fill[c]++] = (int32_t)a;
    }
    for (int64_t i = 0; i < m; ++i) { /* entry (a -> c): c > a, c ascending per row a */
        uint32_t a = (uint32_t)(b->k[i] >> 32), c = (uint32_t)b->k[i];
        ci[fill[a]++] = (int32_t)c;
    }
    free(fill);
    out->n = n; out->nnz = 2 * m; out->row_ptr = rp; out->col_idx = ci;
    return 0;
}

void gg_free(gg_csr *g) {
    if (!g) return;
    free(g->row_ptr); free(g->col_idx);
    g->row_ptr = NULL; g->col_idx = NULL; g->n = 0; g->nnz = 0;
}

/* ------------------------------------------------------------ generators */
static int er_edges(ebuf *b, int32_t n, double p, gg_rng *r) {
    if (p <= 0.0 || n < 2) return 0;
    if (p >= 1.0) {
        for (int32_t v = 1; v < n; ++v)
            for (int32_t w = 0; w < v; ++w)
                if (eb_push(b, (uint32_t)v, (uint32_t)w)) return -1;
        return 0;
    }
    double lp = log(1.0 - p);
    int64_t v = 1, w = -1;
    while (v < n) {
        double u = sm64_unif(r);
        w += 1 + (int64_t)floor(log(1.0 - u) / lp);
        while (w >= v && v < n) { w -= v; v++; }
        if (v < n && eb_push(b, (uint32_t)v, (uint32_t)w)) return -1;
    }
    return 0;
}

int gg_er(int32_t n, double p, uint64_t seed, gg_csr *out) {
    if (n < 0 || !(p >= 0.0) || !out) return -3;
    gg_rng r = {seed};
    ebuf b = {0};
    int rc = er_edges(&b, n, p, &r);
    if (!rc) rc = eb_to_csr(&b, n, out);
    free(b.k);
    return rc;
}

int gg_rmat(int32_t scale, int64_t nsamples, double a, double bq, double c, uint64_t seed,
            gg_csr *out) {
    if (scale < 1 || scale > 30 || nsamples < 0 || !out) return -3;
    gg_rng r = {seed};
    ebuf b = {0};
    double ab = a + bq, abc = a + bq + c;
    for (int64_t s = 0; s < nsamples; ++s) {
        uint32_t u = 0, v = 0;
        for (int32_t l = 0; l < scale; ++l) {
            double x = sm64_unif(&r);
            uint32_t bu, bv;
            if (x < a) { bu = 0; bv = 0; }
            else if (x < ab) { bu = 0; bv = 1; }
            else if (x < abc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu; v = (v << 1) | bv;
        }
        if (eb_push(&b, u, v)) { free(b.k); return -1; }
    }
    int rc = eb_to_csr(&b, (int32_t)1 << scale, out);
    free(b.k);
    return rc;
}

/* Floyd's algorithm: s distinct values from [0,n), returned in `out` (unsorted). */
static int floyd_sample(int32_t n, int32_t s, gg_rng *r, int32_t *out) {
    /* small open-addressing set keyed on the value */
    int32_t cap = 1; while (cap < 4 * s) cap <<= 1;
    int32_t *tab = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    if (!tab) return -1;
    for (int32_t i = 0; i < cap; ++i) tab[i] = -1;
    int32_t cnt = 0;
    for (int32_t j = n - s; j < n; ++j) {
        int32_t t = (int32_t)sm64_below(r, (uint64_t)j + 1);
        /* insert t unless present, else insert j */
        int32_t val = t;
        for (int pass = 0; pass < 2; ++pass) {
            uint32_t h = ((uint32_t)val * 2654435761u) & (uint32_t)(cap - 1);
            int found = 0;
            while (tab[h] != -1) { if (tab[h] == val) { found = 1; break; } h = (h + 1) & (uint32_t)(cap - 1); }
            if (!found) { tab[h] = val; out[cnt++] = val; break; }
            val = j; /* t already taken: take j, which is never present yet */
        }
    }
    free(tab);
    return 0;
}

static int plant_edges(ebuf *b, int32_t n, int32_t nplant, int32_t smin, int32_t smax, gg_rng *r) {
    if (nplant <= 0) return 0;
    if (smin < 2 || smax < smin || smax > n) return -3;
    int32_t *vs = (int32_t *)malloc((size_t)smax * sizeof(int32_t));
    if (!vs) return -1;
    for (int32_t q = 0; q < nplant; ++q) {
        int32_t s = smin + (int32_t)sm64_below(r, (uint64_t)(smax - smin + 1));
        if (floyd_sample(n, s, r, vs)) { free(vs); return -1; }
        for (int32_t i = 0; i < s; ++i)
            for (int32_t j = i + 1; j < s; ++j)
                if (eb_push(b, (uint32_t)vs[i], (uint32_t)vs[j])) { free(vs); return -1; }
    }
    free(vs);
    return 0;
}

/* Solve i0^beta * sum_{i<n} (i+i0)^-beta = target for i0 by bisection (the
 * left side increases with i0). */
static double cl_offset(int32_t n, double beta, double target) {
    double lo = 1e-9, hi = 1e12;
    for (int it = 0; it < 200; ++it) {
        double mid = sqrt(lo * hi);
        double s = 0.0;
        for (int32_t i = 0; i < n; ++i) s += pow(mid / ((double)i + mid), beta);
        if (s < target) lo = mid; else hi = mid;
        if (hi / lo < 1.0 + 1e-12) break;
    }
    return sqrt(lo * hi);
}

/* Chung-Lu: w_i = A (i+i0)^(-1/(gamma-1)), A and i0 chosen so that the mean
 * weight is mean_deg and w_0 = sqrt(sum w) (then every w_i w_j / sum w <= 1
 * and no weight is clamped).  Edge (i,j) appears with probability
 * w_i w_j / sum w.  Then `nplant` cliques of size uniform in [smin,smax]. */
int gg_chung_lu(int32_t n, double gamma, double mean_deg, int32_t nplant, int32_t smin,
                int32_t smax, uint64_t seed, gg_csr *out) {
    if (n < 2 || !(gamma > 1.0) || !(mean_deg > 0.0) || !out) return -3;
    double beta = 1.0 / (gamma - 1.0);
    double W = mean_deg * (double)n;
    double i0 = cl_offset(n, beta, sqrt(W));
    double A = sqrt(W) * pow(i0, beta);
    double *w = (double *)malloc((size_t)n * sizeof(double));
    if (!w) return -1;
    for (int32_t i = 0; i < n; ++i) w[i] = A * pow((double)i + i0, -beta); /* descending */
    gg_rng r = {seed};
    ebuf b = {0};
    for (int32_t u = 0; u < n - 1; ++u) {
        int64_t v = u + 1;
        double p = w[u] * w[v] / W; if (p > 1.0) p = 1.0;
        while (v < n && p > 0.0) {
            if (p != 1.0) {
                double x = sm64_unif(&r);
                v += (int64_t)floor(log(1.0 - x) / log(1.0 - p));
            }
            if (v < n) {
                double q = w[u] * w[v] / W; if (q > 1.0) q = 1.0;
                double x = sm64_unif(&r);
                if (x < q / p && eb_push(&b, (uint32_t)u, (uint32_t)v)) { free(w); free(b.k); return -1; }
                p = q;
                v += 1;
            }
        }
    }
    free(w);
    int rc = plant_edges(&b, n, nplant, smin, smax, &r);
    if (!rc) rc = eb_to_csr(&b, n, out);
    free(b.k);
    return rc;
}

/* G(n,p) plus `nplant` planted cliques (the batched workload's graphs). */
int gg_er_planted(int32_t n, double p, int32_t nplant, int32_t smin, int32_t smax, uint64_t seed,
                  gg_csr *out) {
    if (n < 0 || !(p >= 0.0) || !out) return -3;
    gg_rng r = {seed};
    ebuf b = {0};
    int rc = er_edges(&b, n, p, &r);
    if (!rc) rc = plant_edges(&b, n, nplant, smin, smax, &r);
    if (!rc) rc = eb_to_csr(&b, n, out);
    free(b.k);
    return rc;
}

/* Clean CSR from an edge list; self-loops and duplicates are dropped, the
 * direction of each pair is ignored. */
int gg_from_edges(int32_t n, int64_t ne, const int32_t *src, const int32_t *dst, gg_csr *out) {
    if (n < 0 || ne < 0 || !out) return -3;
    ebuf b = {0};
    for (int64_t i = 0; i < ne; ++i) {
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) { free(b.k); return -3; }
        if (eb_push(&b, (uint32_t)src[i], (uint32_t)dst[i])) { free(b.k); return -1; }
    }
    int rc = eb_to_csr(&b, n, out);
    free(b.k);
    return rc;
}

/* Relabel vertices by a seeded uniform permutation (Fisher-Yates). */
int gg_permute(const gg_csr *in, uint64_t seed, gg_csr *out) {
    if (!in || !out) return -3;
    int32_t n = in->n;
    int32_t *perm = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!perm) return -1;
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    gg_rng r = {seed};
    for (int32_t i = n - 1; i > 0; --i) {
        int32_t j = (int32_t)sm64_below(&r, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    ebuf b = {0};
    for (int32_t u = 0; u < n; ++u)
        for (int32_t p = in->row_ptr[u]; p < in->row_ptr[u + 1]; ++p) {
            int32_t v = in->col_idx[p];
            if (u < v && eb_push(&b, (uint32_t)perm[u], (uint32_t)perm[v])) { free(perm); free(b.k); return -1; }
        }
    free(perm);
    int rc = eb_to_csr(&b, n, out);
    free(b.k);
    return rc;
}
