/*
 * oracle.c -- CPU oracle for exact k-clique counting and listing.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library never
 * links, calls or includes it, and it shares no code, header or table with
 * the GPU path.
 *
 * What it computes, and from which passage of the paper (Wang, Yu, Long,
 * "Efficient k-Clique Listing: An Edge-Oriented Branching Strategy", SIGMOD
 * 2024):
 *
 *  - N_k(G): the number of k-vertex subsets of V that are pairwise adjacent
 *    (Definition of k-clique and the k-clique listing problem, Section 2).
 *    orc_count_vbb follows the vertex-oriented branch-and-bound framework
 *    (Algorithm VBBkC and Eq. vertex-oriented-branching, Section 3) with the
 *    degeneracy vertex ordering used by the VBBkC baselines (Section 7),
 *    recursing on bitsets of the oriented out-neighbourhood.  An optional
 *    shortcut returns C(|P|,l) when the candidate set is itself a clique
 *    (every l-subset of a clique is an l-clique).
 *  - L_k(G): all k-cliques as ascending tuples in lexicographic order.
 *    orc_list_lex is vertex-oriented branching in the natural vertex order
 *    (ascending ids), which emits the tuples directly in lexicographic order.
 *  - orc_count_brute: every k-subset tested pair by pair (n <= 62).
 *  - orc_edge_support: the number of common neighbours of the two endpoints
 *    of every edge (the quantity the truss-based edge ordering minimises,
 *    Section 4.2, Eq. truss-based-edge).
 *  - orc_truss_levelsync: the truss-based edge ordering pi_tau (Section 4.2)
 *    taken level-synchronously -- at level s every remaining edge whose
 *    support is <= s is removed in one round, ranked by (round, edge id),
 *    and each triangle destroyed in that round lowers the support of each of
 *    its surviving edges exactly once.  level(e) is s at removal; tau is the
 *    largest level.  (This is a reading of the sequential greedy rule for
 *    parallel hardware; it keeps the bound |V(g_i)| <= level(e_i) <= tau
 *    behind Eq. tau and the complexity theorem.)
 *  - orc_truss_sequential: the sequential greedy rule of Eq. truss-based-edge
 *    itself (always remove a remaining edge with the fewest common
 *    neighbours; ties by edge id), reporting for every edge its support at
 *    removal.
 *  - orc_degeneracy: degeneracy ordering by repeated removal of a
 *    minimum-degree vertex (ties by id) and the degeneracy delta (Section 1
 *    footnote; Section 7).
 *  - orc_seed_sizes / orc_seed_counts: for a given edge ordering (rank per
 *    edge), the size of the sub-branch g_i of Eq. edge-oriented-branching
 *    at the initial branch, |N(V(e_i), gbar_i)|, and the number of
 *    (k-2)-cliques inside g_i.  Summed over all edges the latter is N_k
 *    (every k-clique is listed exactly once, Section 4.1).
 *
 * Edges are identified by their position in the lexicographic list of pairs
 * (u,v) with u<v.  All counts are uint64; a result that would exceed 2^64-1
 * is reported as ORC_OVERFLOW, never wrapped.
 *
 * Checksums of a listing (a convention of this project; the paper fixes no
 * output order): with sm(x) the SplitMix64 output function of state x
 * (Steele, Lea, Flood 2014), the tuple hash is h = fold of
 * h <- sm(h ^ t_j) over the k ascending entries starting from h = k; the
 * unordered checksum is the sum of h over all tuples and the ordered one is
 * the sum over positions i of sm(h_i ^ sm(i)), both mod 2^64.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_BAD_CSR = -2, ORC_OOM = -3, ORC_BAD_ARG = -4, ORC_OVERFLOW = -6,
       ORC_BUFFER_TOO_SMALL = -5 };

typedef unsigned __int128 u128;

/* --------------------------------------------------------------- basics */

static inline int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* C(n, r) exactly, or ORC_OVERFLOW.  C(n,j) = C(n,j-1) * (n-j+1) / j is an
 * integer at every step, and the 128-bit product cannot overflow while the
 * running value fits 64 bits. */
static int binom(uint64_t n, uint64_t r, uint64_t *out) {
    if (r > n) { *out = 0; return ORC_OK; }
    if (r > n - r) r = n - r;
    u128 c = 1;
    for (uint64_t j = 1; j <= r; ++j) {
        c = c * (u128)(n - r + j) / (u128)j;
        if (c > (u128)UINT64_MAX) return ORC_OVERFLOW;
    }
    *out = (uint64_t)c;
    return ORC_OK;
}

int orc_binom(uint64_t n, uint64_t r, uint64_t *out) { return binom(n, r, out); }

static inline uint64_t sm(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_tuple_hash(const int32_t *t, int32_t k) {
    uint64_t h = (uint64_t)k;
    for (int32_t j = 0; j < k; ++j) h = sm(h ^ (uint64_t)(uint32_t)t[j]);
    return h;
}

/* ------------------------------------------------------------ validation */

/* Input model of Section 2: simple undirected graph.  Rows strictly ascending
 * (no duplicates), no self-loops, ids in range, and symmetric. */
int orc_validate_csr(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci) {
    if (n < 0 || nnz < 0) return ORC_BAD_ARG;
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) return ORC_BAD_CSR;
    for (int32_t u = 0; u < n; ++u) {
        if (rp[u + 1] < rp[u]) return ORC_BAD_CSR;
        for (int32_t p = rp[u]; p < rp[u + 1]; ++p) {
            int32_t v = ci[p];
            if (v < 0 || v >= n || v == u) return ORC_BAD_CSR;
            if (p > rp[u] && ci[p - 1] >= v) return ORC_BAD_CSR;
        }
    }
    for (int32_t u = 0; u < n; ++u)
        for (int32_t p = rp[u]; p < rp[u + 1]; ++p) {
            int32_t v = ci[p];
            if (!bsearch(&u, ci + rp[v], (size_t)(rp[v + 1] - rp[v]), sizeof(int32_t), cmp_i32))
                return ORC_BAD_CSR;
        }
    return ORC_OK;
}

/* ---------------------------------------------------------- edge indexing */

typedef struct {
    int32_t n;
    int64_t m;
    const int32_t *rp, *ci;
    int32_t *ustart; /* first position of row u holding a neighbour > u */
    int64_t *eoff;   /* id of the first edge (u, .) with u < . ; n+1 entries */
    int32_t *eu, *ev;
} edges_t;

static void edges_free(edges_t *E) {
    free(E->ustart); free(E->eoff); free(E->eu); free(E->ev);
}

static int edges_init(edges_t *E, int32_t n, const int32_t *rp, const int32_t *ci) {
    memset(E, 0, sizeof(*E));
    E->n = n; E->rp = rp; E->ci = ci;
    E->ustart = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    E->eoff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!E->ustart || !E->eoff) { edges_free(E); return ORC_OOM; }
    int64_t m = 0;
    for (int32_t u = 0; u < n; ++u) {
        int32_t p = rp[u];
        while (p < rp[u + 1] && ci[p] < u) ++p;
        E->ustart[u] = p;
        E->eoff[u] = m;
        m += rp[u + 1] - p;
    }
    E->eoff[n] = m;
    E->m = m;
    E->eu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    E->ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!E->eu || !E->ev) { edges_free(E); return ORC_OOM; }
    for (int32_t u = 0; u < n; ++u)
        for (int32_t p = E->ustart[u]; p < rp[u + 1]; ++p) {
            int64_t e = E->eoff[u] + (p - E->ustart[u]);
            E->eu[e] = u; E->ev[e] = ci[p];
        }
    return ORC_OK;
}

/* index of key in the sorted array row[0..len), or -1 */
static inline int32_t find_sorted(const int32_t *row, int32_t len, int32_t key) {
    int32_t lo = 0, hi = len;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (row[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < len && row[lo] == key) ? lo : -1;
}

/* id of edge {a,b}, or -1 if absent */
static int64_t edge_id(const edges_t *E, int32_t a, int32_t b) {
    if (a > b) { int32_t t = a; a = b; b = t; }
    int32_t i = find_sorted(E->ci + E->ustart[a], E->rp[a + 1] - E->ustart[a], b);
    return i >= 0 ? E->eoff[a] + i : -1;
}

/* Edge id of every CSR entry (both directions). */
static int64_t *entry_eids(const edges_t *E) {
    int64_t nnz = E->rp[E->n];
    int64_t *pe = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!pe) return NULL;
    for (int32_t x = 0; x < E->n; ++x)
        for (int32_t p = E->rp[x]; p < E->rp[x + 1]; ++p) pe[p] = edge_id(E, x, E->ci[p]);
    return pe;
}

/* The endpoint of edge e whose row is marked ("larger": more neighbours, ties
 * to the larger id) and the one whose row is scanned. */
static inline void split_ends(const edges_t *E, int64_t e, int32_t *big, int32_t *small) {
    int32_t u = E->eu[e], v = E->ev[e];
    int32_t du = E->rp[u + 1] - E->rp[u], dv = E->rp[v + 1] - E->rp[v];
    if (du > dv || (du == dv && u > v)) { *big = u; *small = v; } else { *big = v; *small = u; }
}

int64_t orc_num_edges(int32_t n, const int32_t *rp, const int32_t *ci) {
    int64_t m = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int32_t p = rp[u]; p < rp[u + 1]; ++p) m += ci[p] > u;
    return m;
}

/* Endpoints of every edge, in edge-id order. */
int orc_edge_list(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *eu, int32_t *ev) {
    edges_t E;
    int rc = edges_init(&E, n, rp, ci);
    if (rc) return rc;
    memcpy(eu, E.eu, sizeof(int32_t) * (size_t)E.m);
    memcpy(ev, E.ev, sizeof(int32_t) * (size_t)E.m);
    edges_free(&E);
    return ORC_OK;
}

/* ------------------------------------------------------------ supports */

/* sup(e) = |N(u) cap N(v)|: the larger endpoint's row is marked in a dense
 * array and the smaller endpoint's row is scanned against it. */
int orc_edge_support(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *sup) {
    edges_t E;
    int rc = edges_init(&E, n, rp, ci);
    if (rc) return rc;
    int64_t *pe = entry_eids(&E);
    char *mark = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!pe || !mark) { free(pe); free(mark); edges_free(&E); return ORC_OOM; }
    for (int32_t x = 0; x < n; ++x) {
        for (int32_t p = rp[x]; p < rp[x + 1]; ++p) mark[ci[p]] = 1;
        for (int32_t p = rp[x]; p < rp[x + 1]; ++p) {
            int32_t big, small;
            split_ends(&E, pe[p], &big, &small);
            if (big != x) continue; /* each edge once, from its larger endpoint */
            int32_t c = 0;
            for (int32_t q = rp[small]; q < rp[small + 1]; ++q) c += mark[ci[q]];
            sup[pe[p]] = c;
        }
        for (int32_t p = rp[x]; p < rp[x + 1]; ++p) mark[ci[p]] = 0;
    }
    free(pe); free(mark); edges_free(&E);
    return ORC_OK;
}

/* ------------------------------------------------- truss-based ordering */

/* Level-synchronous truss peel.  Outputs, per edge id: level[e], rank[e]
 * (a permutation of 0..m-1), and optionally the round of removal.  The
 * support array starts from the common-neighbour counts. */
int orc_truss_levelsync(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *level,
                        int32_t *rank, int32_t *round_out, int32_t *n_rounds, int32_t *tau) {
    edges_t E;
    int rc = edges_init(&E, n, rp, ci);
    if (rc) return rc;
    int64_t m = E.m;
    int32_t *sup = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *rnd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1)); /* -1 = alive */
    int64_t *front = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!sup || !rnd || !front) { free(sup); free(rnd); free(front); edges_free(&E); return ORC_OOM; }
    rc = orc_edge_support(n, rp, ci, sup);
    if (rc) { free(sup); free(rnd); free(front); edges_free(&E); return rc; }
    int64_t *pe = entry_eids(&E);
    int64_t *mark = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!pe || !mark) { free(pe); free(mark); free(sup); free(rnd); free(front); edges_free(&E); return ORC_OOM; }
    for (int64_t e = 0; e < m; ++e) rnd[e] = -1;

    /* live[] holds the ids of the remaining edges in ascending order */
    int64_t *live = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!live) { free(sup); free(rnd); free(front); edges_free(&E); return ORC_OOM; }
    int64_t nlive = m;
    for (int64_t e = 0; e < m; ++e) live[e] = e;
    int64_t ranked = 0;
    int32_t s = 0, r = 0, maxlev = 0;
    while (ranked < m) {
        int64_t nf = 0;
        for (int64_t i = 0; i < nlive; ++i)
            if (sup[live[i]] <= s) front[nf++] = live[i];
        if (nf == 0) {
            /* no remaining edge qualifies at this level: go to the next
             * level that has one (empty levels make no round) */
            int32_t mn = INT32_MAX;
            for (int64_t i = 0; i < nlive; ++i)
                if (sup[live[i]] < mn) mn = sup[live[i]];
            s = mn;
            continue;
        }
        /* front[] is in ascending edge-id order */
        for (int64_t i = 0; i < nf; ++i) {
            int64_t e = front[i];
            level[e] = s;
            rank[e] = (int32_t)(ranked + i);
            rnd[e] = r; /* in the frontier of round r */
        }
        if (s > maxlev) maxlev = s;
        /* every triangle of a frontier edge whose two other edges are still
         * present (alive, or in this frontier) is destroyed now; its
         * lowest-id frontier edge lowers each surviving edge once.
         * Triangles of e are found by marking the row of e's larger endpoint
         * (edge ids of its entries) and scanning the smaller one's row. */
        for (int64_t i = 0; i < nf; ++i) {
            int64_t e = front[i];
            int32_t big, small;
            split_ends(&E, e, &big, &small);
            for (int32_t p = rp[big]; p < rp[big + 1]; ++p) mark[ci[p]] = pe[p] + 1;
            for (int32_t q = rp[small]; q < rp[small + 1]; ++q) {
                int64_t f = mark[ci[q]] - 1; /* edge (big, w) */
                if (f < 0) continue;
                int64_t g = pe[q];           /* edge (small, w) */
                int present_f = rnd[f] < 0 || rnd[f] == r;
                int present_g = rnd[g] < 0 || rnd[g] == r;
                if (!present_f || !present_g) continue; /* destroyed in an earlier round */
                int64_t mine = e;
                if (rnd[f] == r && f < mine) mine = f;
                if (rnd[g] == r && g < mine) mine = g;
                if (mine != e) continue;
                if (rnd[f] < 0) sup[f]--;
                if (rnd[g] < 0) sup[g]--;
            }
            for (int32_t p = rp[big]; p < rp[big + 1]; ++p) mark[ci[p]] = 0;
        }
        ranked += nf;
        ++r;
        int64_t j = 0;
        for (int64_t i = 0; i < nlive; ++i)
            if (rnd[live[i]] < 0) live[j++] = live[i];
        nlive = j;
    }
    free(live); free(pe); free(mark);
    if (round_out) memcpy(round_out, rnd, sizeof(int32_t) * (size_t)m);
    if (n_rounds) *n_rounds = r;
    if (tau) *tau = maxlev;
    free(sup); free(rnd); free(front); edges_free(&E);
    return ORC_OK;
}

/* Sequential greedy of Eq. truss-based-edge: repeatedly remove the remaining
 * edge with the fewest common neighbours in the remaining graph (ties: lowest
 * edge id).  order[i] = id of the i-th removed edge, peel[e] = its number of
 * common neighbours at removal.  O(m^2) scan; meant for small graphs. */
int orc_truss_sequential(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *order,
                         int32_t *peel) {
    edges_t E;
    int rc = edges_init(&E, n, rp, ci);
    if (rc) return rc;
    int64_t m = E.m;
    int32_t *sup = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    char *gone = (char *)calloc((size_t)(m > 0 ? m : 1), 1);
    if (!sup || !gone) { free(sup); free(gone); edges_free(&E); return ORC_OOM; }
    orc_edge_support(n, rp, ci, sup);
    for (int64_t i = 0; i < m; ++i) {
        int64_t best = -1;
        for (int64_t e = 0; e < m; ++e)
            if (!gone[e] && (best < 0 || sup[e] < sup[best])) best = e;
        order[i] = (int32_t)best;
        peel[best] = sup[best];
        gone[best] = 1;
        int32_t u = E.eu[best], v = E.ev[best];
        int32_t a = rp[u], b = rp[v];
        while (a < rp[u + 1] && b < rp[v + 1]) {
            if (ci[a] < ci[b]) { ++a; continue; }
            if (ci[a] > ci[b]) { ++b; continue; }
            int32_t w = ci[a]; ++a; ++b;
            int64_t f = edge_id(&E, u, w), g = edge_id(&E, v, w);
            if (gone[f] || gone[g]) continue;
            sup[f]--; sup[g]--;
        }
    }
    free(sup); free(gone); edges_free(&E);
    return ORC_OK;
}

/* ---------------------------------------------------- degeneracy order */

/* Repeatedly remove a vertex of minimum remaining degree, ties to the
 * smaller id (binary heap keyed by (degree, id) with lazy deletion).
 * order[i] = i-th removed vertex; delta = largest degree seen at removal. */
typedef struct { int32_t d, v; } hent;
static inline int hless(hent a, hent b) { return a.d < b.d || (a.d == b.d && a.v < b.v); }

int orc_degeneracy(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *order, int32_t *delta) {
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    char *gone = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t cap = (int64_t)n + rp[n] + 1;
    hent *h = (hent *)malloc(sizeof(hent) * (size_t)cap);
    if (!deg || !gone || !h) { free(deg); free(gone); free(h); return ORC_OOM; }
    int64_t hs = 0;
#define HPUSH(x) do { int64_t i_ = hs++; h[i_] = (x); \
    while (i_ > 0 && hless(h[i_], h[(i_ - 1) / 2])) { hent t_ = h[i_]; h[i_] = h[(i_ - 1) / 2]; h[(i_ - 1) / 2] = t_; i_ = (i_ - 1) / 2; } } while (0)
    for (int32_t v = 0; v < n; ++v) { deg[v] = rp[v + 1] - rp[v]; hent x = {deg[v], v}; HPUSH(x); }
    int32_t d = 0, cnt = 0;
    while (cnt < n) {
        hent top = h[0];
        h[0] = h[--hs];
        int64_t i = 0;
        for (;;) {
            int64_t l = 2 * i + 1, r = l + 1, s = i;
            if (l < hs && hless(h[l], h[s])) s = l;
            if (r < hs && hless(h[r], h[s])) s = r;
            if (s == i) break;
            hent t = h[i]; h[i] = h[s]; h[s] = t; i = s;
        }
        if (gone[top.v] || top.d != deg[top.v]) continue; /* stale entry */
        gone[top.v] = 1;
        order[cnt++] = top.v;
        if (top.d > d) d = top.d;
        for (int32_t p = rp[top.v]; p < rp[top.v + 1]; ++p) {
            int32_t w = ci[p];
            if (!gone[w]) { deg[w]--; hent x = {deg[w], w}; HPUSH(x); }
        }
    }
#undef HPUSH
    if (delta) *delta = d;
    free(deg); free(gone); free(h);
    return ORC_OK;
}

/* ------------------------------------------- VBB counting on bitsets */

/* Shared state of one counting run (degeneracy-ordered VBB). */
typedef struct {
    int32_t n, k, shortcut;
    const int32_t *rp, *ci;
    const int32_t *pos;   /* pos[v] = index of v in the degeneracy order */
    const int32_t *roots; /* root vertices to expand */
    int64_t nroots;
    int32_t maxout;       /* max |N+(v)| */
    atomic_long next;     /* next root (dynamic chunks) */
    atomic_int fail;
    uint64_t total;
    pthread_mutex_t mu;
} vbb_t;

static inline int pc64(uint64_t x) { return __builtin_popcountll(x); }

/* count(P, l) of Algorithm VBBkC on a local oriented adjacency A+ (rows of W
 * words, bit j of row i set iff local vertices i<j are adjacent).  P is a
 * bitset over local ids.  Returns 0 or ORC_OVERFLOW. */
static int vbb_rec(const uint64_t *A, int W, const uint64_t *P, int l, int shortcut,
                   uint64_t *scratch, uint64_t *out) {
    int size = 0;
    for (int w = 0; w < W; ++w) size += pc64(P[w]);
    if (size < l) { *out = 0; return ORC_OK; }
    if (l == 1) { *out = (uint64_t)size; return ORC_OK; }
    if (l == 2) {
        uint64_t s = 0;
        for (int w = 0; w < W; ++w)
            for (uint64_t b = P[w]; b; b &= b - 1) {
                int x = w * 64 + __builtin_ctzll(b);
                for (int q = 0; q < W; ++q) s += (uint64_t)pc64(A[x * W + q] & P[q]);
            }
        *out = s;
        return ORC_OK;
    }
    if (shortcut) {
        /* P is a clique iff every member is adjacent to all later members */
        int later = size, clique = 1;
        for (int w = 0; w < W && clique; ++w)
            for (uint64_t b = P[w]; b; b &= b - 1) {
                int x = w * 64 + __builtin_ctzll(b);
                int d = 0;
                for (int q = 0; q < W; ++q) d += pc64(A[x * W + q] & P[q]);
                --later;
                if (d != later) { clique = 0; break; }
            }
        if (clique) return binom((uint64_t)size, (uint64_t)l, out);
    }
    uint64_t s = 0;
    uint64_t *child = scratch;
    for (int w = 0; w < W; ++w)
        for (uint64_t b = P[w]; b; b &= b - 1) {
            int x = w * 64 + __builtin_ctzll(b);
            for (int q = 0; q < W; ++q) child[q] = A[x * W + q] & P[q];
            uint64_t c;
            int rc = vbb_rec(A, W, child, l - 1, shortcut, scratch + W, &c);
            if (rc) return rc;
            if (__builtin_add_overflow(s, c, &s)) return ORC_OVERFLOW;
        }
    *out = s;
    return ORC_OK;
}

static void *vbb_worker(void *arg) {
    vbb_t *S = (vbb_t *)arg;
    int32_t n = S->n, k = S->k;
    int Wmax = (S->maxout + 63) / 64 + 1;
    int32_t *loc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(S->maxout + 1));
    uint64_t *A = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(S->maxout + 1) * (size_t)Wmax);
    uint64_t *scratch = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(k + 2) * (size_t)Wmax);
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint64_t acc = 0;
    if (!loc || !A || !scratch || !mark) { atomic_store(&S->fail, ORC_OOM); goto done; }
    for (int32_t i = 0; i < n; ++i) mark[i] = -1;
    for (;;) {
        long r0 = atomic_fetch_add(&S->next, 16);
        if (r0 >= S->nroots || atomic_load(&S->fail)) break;
        long r1 = r0 + 16 < S->nroots ? r0 + 16 : S->nroots;
        for (long ri = r0; ri < r1; ++ri) {
            int32_t v = S->roots[ri];
            /* out-neighbours of v in the degeneracy order, sorted by order */
            int32_t c = 0;
            for (int32_t p = S->rp[v]; p < S->rp[v + 1]; ++p)
                if (S->pos[S->ci[p]] > S->pos[v]) loc[c++] = S->ci[p];
            if (c < k - 1) continue;
            /* insertion sort by degeneracy position (c <= delta) */
            for (int32_t i = 1; i < c; ++i) {
                int32_t x = loc[i], j = i - 1;
                while (j >= 0 && S->pos[loc[j]] > S->pos[x]) { loc[j + 1] = loc[j]; --j; }
                loc[j + 1] = x;
            }
            int W = (c + 63) / 64;
            for (int32_t i = 0; i < c; ++i) mark[loc[i]] = i;
            memset(A, 0, sizeof(uint64_t) * (size_t)c * (size_t)W);
            for (int32_t i = 0; i < c; ++i) {
                int32_t x = loc[i];
                for (int32_t p = S->rp[x]; p < S->rp[x + 1]; ++p) {
                    int32_t j = mark[S->ci[p]];
                    if (j > i) A[i * W + j / 64] |= 1ULL << (j % 64);
                }
            }
            for (int32_t i = 0; i < c; ++i) mark[loc[i]] = -1;
            uint64_t *P = scratch;
            memset(P, 0, sizeof(uint64_t) * (size_t)W);
            for (int32_t i = 0; i < c; ++i) P[i / 64] |= 1ULL << (i % 64);
            uint64_t cnt;
            int rc = vbb_rec(A, W, P, k - 1, S->shortcut, scratch + W, &cnt);
            if (rc || __builtin_add_overflow(acc, cnt, &acc)) {
                atomic_store(&S->fail, rc ? rc : ORC_OVERFLOW);
                goto done;
            }
        }
    }
done:
    pthread_mutex_lock(&S->mu);
    if (__builtin_add_overflow(S->total, acc, &S->total)) atomic_store(&S->fail, ORC_OVERFLOW);
    pthread_mutex_unlock(&S->mu);
    free(loc); free(A); free(scratch); free(mark);
    return NULL;
}

/* Run the degeneracy-ordered VBB over the root vertices order[r_begin..r_end)
 * of the degeneracy order (all roots: N_k). */
static int vbb_run(int32_t n, const int32_t *rp, const int32_t *ci, int32_t k, int32_t nthreads,
                   int32_t shortcut, int64_t r_begin, int64_t r_end, uint64_t *out) {
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!order || !pos) { free(order); free(pos); return ORC_OOM; }
    int32_t delta;
    int rc = orc_degeneracy(n, rp, ci, order, &delta);
    if (rc) { free(order); free(pos); return rc; }
    for (int32_t i = 0; i < n; ++i) pos[order[i]] = i;
    if (r_begin < 0) r_begin = 0;
    if (r_end > n) r_end = n;
    if (r_end < r_begin) r_end = r_begin;
    vbb_t S;
    memset(&S, 0, sizeof(S));
    S.n = n; S.k = k; S.shortcut = shortcut; S.rp = rp; S.ci = ci; S.pos = pos;
    S.roots = order + r_begin; S.nroots = r_end - r_begin;
    S.maxout = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t c = 0;
        for (int32_t p = rp[v]; p < rp[v + 1]; ++p) c += pos[ci[p]] > pos[v];
        if (c > S.maxout) S.maxout = c;
    }
    atomic_init(&S.next, 0);
    atomic_init(&S.fail, 0);
    pthread_mutex_init(&S.mu, NULL);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, vbb_worker, &S);
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&S.mu);
    rc = atomic_load(&S.fail);
    if (!rc) *out = S.total;
    free(order); free(pos);
    return rc;
}

/* N_k by degeneracy-ordered VBB.  k=1 -> n, k=2 -> m (the l=1 / l=2
 * terminations of the framework). */
int orc_count_vbb(int32_t n, const int32_t *rp, const int32_t *ci, int32_t k, int32_t nthreads,
                  int32_t shortcut, uint64_t *out) {
    if (k < 1 || nthreads < 1) return ORC_BAD_ARG;
    if (k == 1) { *out = (uint64_t)n; return ORC_OK; }
    if (k == 2) { *out = (uint64_t)orc_num_edges(n, rp, ci); return ORC_OK; }
    return vbb_run(n, rp, ci, k, nthreads, shortcut, 0, n, out);
}

/* ----------------------------------------------------- brute force */

/* Every k-subset of V (n <= 62), each tested on all of its pairs. */
int orc_count_brute(int32_t n, const int32_t *rp, const int32_t *ci, int32_t k, uint64_t *out) {
    if (n > 62 || k < 1) return ORC_BAD_ARG;
    if (k > n) { *out = 0; return ORC_OK; }
    uint64_t adj[62];
    for (int32_t u = 0; u < n; ++u) {
        adj[u] = 0;
        for (int32_t p = rp[u]; p < rp[u + 1]; ++p) adj[u] |= 1ULL << ci[p];
    }
    uint64_t cnt = 0;
    uint64_t s = (k == 64) ? ~0ULL : ((1ULL << k) - 1);
    uint64_t lim = 1ULL << n;
    while (s < lim) {
        int ok = 1;
        for (uint64_t b = s; b && ok; b &= b - 1) {
            int u = __builtin_ctzll(b);
            uint64_t others = s & ~(1ULL << u);
            if ((adj[u] & others) != others) ok = 0;
        }
        cnt += (uint64_t)ok;
        /* next subset with the same popcount (Gosper) */
        uint64_t c = s & -s, r = s + c;
        if (r == 0) break;
        s = (((r ^ s) >> 2) / c) | r;
    }
    *out = cnt;
    return ORC_OK;
}

/* ------------------------------------------- lexicographic listing */

typedef struct {
    int32_t n, k;
    const int32_t *rp, *ci;
    const int32_t *up;        /* first position of row v holding a neighbour > v */
    const uint64_t *base;     /* per-root first global position (pass 2), or NULL */
    uint64_t *per_root;       /* per-root count (pass 1) */
    int32_t *buf;             /* output tuples (pass 2), or NULL */
    uint64_t cap;
    atomic_long next;
    atomic_int fail;
    uint64_t h_ord, h_unord;
    pthread_mutex_t mu;
} lex_t;

typedef struct {
    int32_t *cand;   /* k levels x n candidates */
    int64_t *stamp;  /* k levels x n membership stamps */
    int64_t tick;
    int32_t S[64];
    uint64_t count, pos, ho, hu;
} lexw_t;

/* Natural-order vertex branching: candidates P (ascending ids, all larger
 * than the last chosen vertex), l vertices still to choose.  Children are
 * taken in ascending order, so tuples come out in lexicographic order. */
static int lex_rec(lex_t *L, lexw_t *T, const int32_t *P, int32_t np, int depth, int l) {
    int32_t n = L->n;
    if (np < l) return ORC_OK;
    if (l == 1) {
        for (int32_t i = 0; i < np; ++i) {
            T->S[depth] = P[i];
            if (L->base) {
                uint64_t h = orc_tuple_hash(T->S, L->k);
                T->hu += h;
                T->ho += sm(h ^ sm(T->pos));
                if (L->buf) memcpy(L->buf + T->pos * (uint64_t)L->k, T->S, sizeof(int32_t) * (size_t)L->k);
                T->pos++;
            }
            if (__builtin_add_overflow(T->count, 1, &T->count)) return ORC_OVERFLOW;
        }
        return ORC_OK;
    }
    int64_t *st = T->stamp + (size_t)depth * n;
    int64_t tick = ++T->tick;
    for (int32_t i = 0; i < np; ++i) st[P[i]] = tick;
    int32_t *child = T->cand + (size_t)(depth + 1) * n;
    for (int32_t i = 0; np - i >= l; ++i) {
        int32_t x = P[i];
        T->S[depth] = x;
        int32_t nc = 0;
        for (int32_t p = L->up[x]; p < L->rp[x + 1]; ++p)
            if (st[L->ci[p]] == tick) child[nc++] = L->ci[p];
        int rc = lex_rec(L, T, child, nc, depth + 1, l - 1);
        if (rc) return rc;
        /* the child's stamps live at depth+1; ours are untouched */
    }
    return ORC_OK;
}

static void *lex_worker(void *arg) {
    lex_t *L = (lex_t *)arg;
    int32_t n = L->n, k = L->k;
    lexw_t T;
    memset(&T, 0, sizeof(T));
    T.cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1) * (size_t)(n > 0 ? n : 1));
    T.stamp = (int64_t *)calloc((size_t)(k + 1) * (size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!T.cand || !T.stamp) { atomic_store(&L->fail, ORC_OOM); goto done; }
    for (;;) {
        long v = atomic_fetch_add(&L->next, 1);
        if (v >= n || atomic_load(&L->fail)) break;
        T.S[0] = (int32_t)v;
        T.count = 0;
        if (L->base) T.pos = L->base[v];
        int32_t np = 0;
        for (int32_t p = L->up[v]; p < L->rp[v + 1]; ++p) T.cand[np++] = L->ci[p];
        int rc;
        if (k == 1) {
            T.count = 1;
            if (L->base) {
                uint64_t h = orc_tuple_hash(T.S, 1);
                T.hu += h; T.ho += sm(h ^ sm(T.pos));
                if (L->buf) L->buf[T.pos] = (int32_t)v;
            }
            rc = ORC_OK;
        } else {
            rc = lex_rec(L, &T, T.cand, np, 1, k - 1);
        }
        if (rc) { atomic_store(&L->fail, rc); break; }
        L->per_root[v] = T.count;
    }
done:
    pthread_mutex_lock(&L->mu);
    L->h_ord += T.ho; L->h_unord += T.hu;
    pthread_mutex_unlock(&L->mu);
    free(T.cand); free(T.stamp);
    return NULL;
}

static int lex_run(lex_t *L, int32_t nthreads) {
    atomic_init(&L->next, 0);
    atomic_init(&L->fail, 0);
    pthread_mutex_init(&L->mu, NULL);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int32_t t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, lex_worker, L);
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&L->mu);
    return atomic_load(&L->fail);
}

/* All k-cliques in lexicographic order of ascending tuples.  Always returns
 * the count and both checksums; writes the tuples to buf (count*k int32)
 * when buf is non-NULL and cap >= count, else returns ORC_BUFFER_TOO_SMALL
 * with *count set. */
int orc_list_lex(int32_t n, const int32_t *rp, const int32_t *ci, int32_t k, int32_t nthreads,
                 int32_t *buf, uint64_t cap, uint64_t *count, uint64_t *h_ord, uint64_t *h_unord) {
    if (k < 1 || k > 64 || nthreads < 1) return ORC_BAD_ARG;
    int32_t *up = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    uint64_t *per = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    uint64_t *base = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n + 1));
    if (!up || !per || !base) { free(up); free(per); free(base); return ORC_OOM; }
    for (int32_t v = 0; v < n; ++v) {
        int32_t p = rp[v];
        while (p < rp[v + 1] && ci[p] < v) ++p;
        up[v] = p;
    }
    lex_t L;
    memset(&L, 0, sizeof(L));
    L.n = n; L.k = k; L.rp = rp; L.ci = ci; L.up = up; L.per_root = per;
    int rc = lex_run(&L, nthreads); /* pass 1: counts per smallest vertex */
    uint64_t tot = 0;
    for (int32_t v = 0; v < n && !rc; ++v) {
        base[v] = tot;
        if (__builtin_add_overflow(tot, per[v], &tot)) rc = ORC_OVERFLOW;
    }
    if (!rc) {
        *count = tot;
        if (buf && cap < tot) rc = ORC_BUFFER_TOO_SMALL;
    }
    if (!rc) {
        memset(&L, 0, sizeof(L));
        L.n = n; L.k = k; L.rp = rp; L.ci = ci; L.up = up; L.per_root = per; L.base = base;
        L.buf = buf; L.cap = cap;
        rc = lex_run(&L, nthreads); /* pass 2: positions, checksums, tuples */
        if (!rc) { *h_ord = L.h_ord; *h_unord = L.h_unord; }
    }
    free(up); free(per); free(base);
    return rc;
}

/* ------------------------------------------ sub-branches of an ordering */

/* For every edge e_i = (u,v) with rank r: the vertex set of g_i in Eq.
 * edge-oriented-branching at the initial branch, i.e. the w adjacent to both
 * u and v through edges ranked after e_i.  Writes |V(g_i)| per edge id. */
int orc_seed_sizes(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *rank,
                   int32_t *csize) {
    edges_t E;
    int rc = edges_init(&E, n, rp, ci);
    if (rc) return rc;
    int64_t *pe = entry_eids(&E);
    int64_t *mark = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!pe || !mark) { free(pe); free(mark); edges_free(&E); return ORC_OOM; }
    for (int32_t x = 0; x < n; ++x) {
        for (int32_t p = rp[x]; p < rp[x + 1]; ++p) mark[ci[p]] = pe[p] + 1;
        for (int32_t p = rp[x]; p < rp[x + 1]; ++p) {
            int64_t e = pe[p];
            int32_t big, small;
            split_ends(&E, e, &big, &small);
            if (big != x) continue;
            int32_t c = 0;
            for (int32_t q = rp[small]; q < rp[small + 1]; ++q) {
                int64_t f = mark[ci[q]] - 1;
                if (f >= 0 && rank[f] > rank[e] && rank[pe[q]] > rank[e]) ++c;
            }
            csize[e] = c;
        }
        for (int32_t p = rp[x]; p < rp[x + 1]; ++p) mark[ci[p]] = 0;
    }
    free(pe); free(mark); edges_free(&E);
    return ORC_OK;
}

/* Number of l-cliques in a small graph given as strictly-upper adjacency
 * lists over local ids 0..c-1 (plain recursion, ascending extension). */
static int small_cliques(const uint64_t *A, int W, const uint64_t *P, int l, uint64_t *scratch,
                         uint64_t *out) {
    return vbb_rec(A, W, P, l, 1, scratch, out);
}

/* For the listed edge ids: number of (k-2)-cliques of g_i (vertices as in
 * orc_seed_sizes, edges = pairs among them whose own rank is after e_i).
 * k >= 3. */
int orc_seed_counts(int32_t n, const int32_t *rp, const int32_t *ci, const int32_t *rank,
                    int32_t k, const int64_t *eids, int64_t ne, uint64_t *out) {
    if (k < 3) return ORC_BAD_ARG;
    edges_t E;
    int rc = edges_init(&E, n, rp, ci);
    if (rc) return rc;
    int32_t cap = 0;
    for (int32_t v = 0; v < n; ++v) if (rp[v + 1] - rp[v] > cap) cap = rp[v + 1] - rp[v];
    int Wmax = (cap + 63) / 64 + 1;
    int32_t *C = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    uint64_t *A = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap + 1) * (size_t)Wmax);
    uint64_t *scratch = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(k + 2) * (size_t)Wmax);
    if (!C || !A || !scratch) { free(C); free(A); free(scratch); edges_free(&E); return ORC_OOM; }
    for (int64_t q = 0; q < ne && !rc; ++q) {
        int64_t e = eids[q];
        if (e < 0 || e >= E.m) { rc = ORC_BAD_ARG; break; }
        int32_t u = E.eu[e], v = E.ev[e], c = 0, re = rank[e];
        if (rp[u + 1] - rp[u] > rp[v + 1] - rp[v]) { int32_t t = u; u = v; v = t; }
        for (int32_t a = rp[u]; a < rp[u + 1]; ++a) { /* ascending w */
            int32_t w = ci[a];
            if (rank[edge_id(&E, u, w)] <= re) continue;
            int64_t g = edge_id(&E, v, w);
            if (g >= 0 && rank[g] > re) C[c++] = w;
        }
        if (k == 3) { out[q] = (uint64_t)c; continue; }
        int W = (c + 63) / 64;
        if (W == 0) { out[q] = 0; continue; }
        memset(A, 0, sizeof(uint64_t) * (size_t)c * (size_t)W);
        for (int32_t i = 0; i < c; ++i)
            for (int32_t j = i + 1; j < c; ++j) {
                int64_t f = edge_id(&E, C[i], C[j]);
                if (f >= 0 && rank[f] > re) A[i * W + j / 64] |= 1ULL << (j % 64);
            }
        uint64_t *P = scratch;
        memset(P, 0, sizeof(uint64_t) * (size_t)W);
        for (int32_t i = 0; i < c; ++i) P[i / 64] |= 1ULL << (i % 64);
        rc = small_cliques(A, W, P, k - 2, scratch + W, &out[q]);
    }
    free(C); free(A); free(scratch); edges_free(&E);
    return rc;
}
