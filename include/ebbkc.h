/*
 * ebbkc.h -- exact k-clique counting and listing on one MI355X (gfx950).
 *
 * The method is EBBkC (Wang, Yu, Long, "Efficient k-Clique Listing: An
 * Edge-Oriented Branching Strategy", SIGMOD 2024) in its hybrid form
 * EBBkC-H with early termination (Section 4.4 and Section 5):
 *
 *   1. ebbkc_prepare computes the truss-based edge ordering pi_tau of the
 *      input graph (Section 4.2, Eq. truss-based-edge), taken
 *      level-synchronously: at level s every remaining edge with at most s
 *      common neighbours in the remaining graph is removed in one round and
 *      ranked by (round, edge id).  level(e) is the s at which e is removed
 *      and tau is the largest level (Eq. tau bounds every sub-branch size by
 *      it).  The ranks are stored next to the adjacency.
 *   2. ebbkc_count / ebbkc_list branch on every edge e_i = (u,v) in that
 *      order (Eq. edge-oriented-branching): the sub-branch graph g_i has the
 *      common neighbours of u and v through edges ranked after e_i, and the
 *      edges among them ranked after e_i.  g_i is coloured greedily, ordered
 *      by non-increasing colour, oriented into a DAG, and searched with
 *      pruning Rules (1) and (2) of Section 4.3; a candidate set that is a
 *      clique, a 2-plex or (per the t rule of Section 6.1) a 3-plex is
 *      finished in closed form (Section 5, Algorithms kC2Plex, kCtPlex).
 *
 * ebbkc_options.ordering selects the paper's other variants on the same
 * engine instead (EBBkC-C, EBBkC-T, and VBBkC's edge- and node-parallel
 * schemes); every variant gives the same counts and listings.
 *
 * Conventions
 *   - The graph is simple and undirected (Section 2), given as int32 CSR
 *     with both directions stored, rows strictly ascending, no self-loops.
 *     ebbkc_prepare rejects anything else with EBBKC_E_BAD_CSR.
 *   - An edge id is the position of the pair (u,v), u<v, in lexicographic
 *     order.  Vertex ids are the CSR row indices.
 *   - Every call is ordered on the given HIP stream (NULL = the null
 *     stream); calls that return host values synchronise that stream first.
 *   - Every call returns an ebbkc_status; nothing is thrown across this
 *     boundary.  Outputs are written only on EBBKC_OK, except where a
 *     function says otherwise.
 *   - Counts are exact: a true count of 2^64 or more is reported as
 *     EBBKC_E_OVERFLOW, never as a wrapped value.
 *   - A handle must not be used by two calls at the same time.
 */
#ifndef EBBKC_H
#define EBBKC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ebbkc_graph ebbkc_graph; /* opaque; owns its device memory */

typedef enum {
    EBBKC_OK = 0,
    EBBKC_E_INVALID_ARG = -1,
    EBBKC_E_BAD_CSR = -2,          /* input is not a simple undirected CSR */
    EBBKC_E_OOM = -3,              /* device memory exhausted */
    EBBKC_E_K_RANGE = -4,          /* k < 1 */
    EBBKC_E_BUFFER_TOO_SMALL = -5, /* listing buffer smaller than the result */
    EBBKC_E_OVERFLOW = -6,         /* exact count does not fit 64 bits */
    EBBKC_E_WIDTH = -7,            /* a sub-branch exceeds the widest bitmap class */
    EBBKC_E_HIP = -8,              /* a HIP runtime call failed */
    EBBKC_E_CANCELLED = -9,        /* a served request withdrawn by ebbkc_server_cancel */
    EBBKC_E_SCRATCH = -10          /* ebbkc_count_noalloc: the count needs more than its fixed
                                      256 MiB scratch */
} ebbkc_status;

enum { EBBKC_PTR_HOST = 0, EBBKC_PTR_DEVICE = 1 };

/* Tuning and ablation switches.  ebbkc_default_options fills the defaults;
 * no switch changes any count or listing. */
typedef struct {
    int32_t early_termination; /* 1 (default): clique / 2-plex closed forms (Section 5) */
    int32_t t_plex;            /* largest t whose t-plexes (every vertex misses at most t-1
                                  others) end the branching early (Section 5): 1 cliques, 2 also
                                  2-plexes (Algorithm kC2Plex, closed form), 3 also 3-plexes
                                  (their missing pairs form paths and cycles: closed form), 4..16
                                  also t-plexes by Algorithm kCtPlex (branching on the inverse
                                  graph, the vertices adjacent to all others in closed form; for
                                  counts of at most 96 vertices); 0 (default) the rule of Section
                                  6.1: 2 when k <= tau/2, else 3.  Other values: E_INVALID_ARG
                                  from ebbkc_prepare.  Listings branch beyond t = 2. */
    int32_t rule1;             /* 1 (default): colour pruning Rule (1), Section 4.3 */
    int32_t rule2;             /* 1 (default): colour pruning Rule (2), Section 4.3 */
    int32_t waves_per_block;   /* workgroup size in wavefronts (default 4) */
    int32_t blocks_per_cu;     /* persistent workgroups per compute unit (0 = as many as fit;
                                  -1 = one workgroup per four tasks, not persistent; -2 = one fewer
                                  than fit, so launches on other streams always find room) */
    int32_t split_threshold;   /* root-branch work above which a seed is split (0 = auto, <0 = never) */
    int32_t count_work;        /* 1: record search work counters (ebbkc_last_work); default 0 */
    int32_t dense_k4;          /* 4-cliques of a dense candidate set counted from its missing pairs
                                  when that costs less than branching: weight (percent) of its cost
                                  estimate, 0 = default (100), < 0 = never */
    int32_t ordering;          /* edge order of the initial branch and colouring below it:
                                  EBBKC_ORDER_HYBRID (0, default): truss-based order at the
                                    initial branch, each g_i coloured on its own (EBBkC-H,
                                    Section 4.4);
                                  EBBKC_ORDER_COLOR (1): one greedy colouring of G, vertices by
                                    non-increasing colour, edges in the lexicographic order of
                                    their endpoints' positions; every g_i keeps G's colours
                                    (EBBkC-C, Section 4.3);
                                  EBBKC_ORDER_DEGEN_VERTEX (2): vertices in a degeneracy order,
                                    edges in the lexicographic order of their endpoints'
                                    positions, each g_i coloured on its own: vertex-oriented
                                    branching (Algorithm VBBkC, degeneracy order) with its first
                                    two steps taken together, the edge-parallel scheme of
                                    Section 6.2 (7);
                                  EBBKC_ORDER_TRUSS (3): the truss-based order at every level
                                    (EBBkC-T, Section 4.2): size pruning and the clique / 2-plex
                                    terminations, no colour rules; k <= 99.  It applies to the
                                    counting calls; listings and batches under it use the
                                    colour order below the initial branch (same result).
                                  EBBKC_ORDER_DEGEN_VERTEX_NP (4): the same vertex order and
                                    edge ranks as DEGEN_VERTEX, but a whole-graph count takes one
                                    root per vertex v, G[N+(v)] (the node-parallel scheme of
                                    Section 6.2 (7)); |N+(v)| <= 256 or EBBKC_E_WIDTH.  Rank ranges,
                                    per-seed counts, listings and batches under it use the edge
                                    roots of DEGEN_VERTEX (same results).
                                  Other values: EBBKC_E_INVALID_ARG. */
    int32_t batch_build;       /* batches (ebbkc_batch_create): where each task's sub-branch comes
                                  from.  EBBKC_BATCH_ARENA (1): every graph's sub-branch arena is
                                  built in device memory once and tasks load their g_i from it;
                                  EBBKC_BATCH_BUILD (2): no arena, every task builds its g_i in
                                  LDS from the graph's arrays (memory O(m) per graph, for batches
                                  whose arenas would not fit); 0 (default): arenas when every
                                  graph already has one or their total size is at most half the
                                  free device memory, else build.  Counts are the same. */
    int32_t node_split;        /* runtime splitting of search nodes over waves through a device
                                  queue (root sub-branches and their subtrees are independent,
                                  Section 6.2 (7)): 0 (default): a node with l >= 4 and at least
                                  2^20 l-subsets is handed to a waiting wave while some wave waits
                                  for work; n >= 2: the same with n l-subsets; 1: every node with
                                  l >= 4 is handed over while the queue has room (exercises the
                                  queue at every depth); -1: off.  Not used by listings, per-seed
                                  counts, EBBkC-T, non-persistent launches (blocks_per_cu = -1)
                                  or served epochs (they run concurrently, and waves waiting for
                                  nodes would hold compute units the other epochs need).  Counts
                                  are the same. */
    int32_t adj_max_n;         /* sub-branch builds (Eq. edge-oriented-branching: the edges among
                                  V(g_i) ranked after e_i): graphs with at most this many vertices
                                  get an adjacency bitmap of G at prepare (n^2 / 8 bytes plus a
                                  quarter of that), and every pair of V(g_i) is tested against it
                                  (about |V(g_i)|^2 / 2 tests instead of a scan of every member's
                                  row); larger graphs scan.  0 (default): 8192; -1: never; at most
                                  32768, else EBBKC_E_INVALID_ARG.  Counts are the same. */
    int32_t reserved[2];
} ebbkc_options;

enum { EBBKC_BATCH_AUTO = 0, EBBKC_BATCH_ARENA = 1, EBBKC_BATCH_BUILD = 2 };

enum {
    EBBKC_ORDER_HYBRID = 0,
    EBBKC_ORDER_COLOR = 1,
    EBBKC_ORDER_DEGEN_VERTEX = 2,
    EBBKC_ORDER_TRUSS = 3,
    EBBKC_ORDER_DEGEN_VERTEX_NP = 4
};

typedef struct {
    int32_t n;          /* vertices */
    int64_t m;          /* undirected edges */
    int32_t tau;        /* largest truss level (max sub-branch size bound) */
    int32_t rounds;     /* peel rounds */
    int32_t max_degree;
    int64_t device_bytes; /* device memory held by the handle */
    double prepare_ms;    /* device time of the last ebbkc_prepare */
} ebbkc_info;

enum {
    EBBKC_LIST_SORTED = 1 /* sort the written tuples lexicographically */
};

/* Array selectors for ebbkc_export. */
enum {
    EBBKC_ARR_SUPPORT = 0, /* int32[m]: common neighbours of each edge in G */
    EBBKC_ARR_RANK = 1,    /* int32[m]: position of each edge in the initial branch's edge order
                              (pi_tau under the default ordering) */
    EBBKC_ARR_LEVEL = 2,   /* int32[m]: truss level of each edge */
    EBBKC_ARR_SUBSIZE = 3, /* int32[m]: |V(g_i)| of each edge's sub-branch */
    EBBKC_ARR_VERTEX_POS = 4,   /* int32[n]: position of each vertex in the vertex order the
                                   edge ranks follow (orderings COLOR, DEGEN_VERTEX and
                                   DEGEN_VERTEX_NP only) */
    EBBKC_ARR_VERTEX_COLOR = 5  /* int32[n]: colour (1, 2, ...) of each vertex in the greedy
                                   colouring of G (ordering COLOR only) */
};

void ebbkc_default_options(ebbkc_options *opt);

/* Build a handle for the graph: validate the CSR, copy it to the device
 * (ptr_kind says where row_ptr/col_idx live), compute supports, the
 * level-synchronous truss ordering, ranks and the rank-tagged adjacency.
 * row_ptr: n+1 int32; col_idx: nnz int32 (nnz = 2m).  The caller keeps
 * ownership of the input arrays; they may be freed when this returns.
 * opt may be NULL (defaults).  On success *out owns the handle. */
ebbkc_status ebbkc_prepare(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int64_t nnz,
                           int32_t ptr_kind, const ebbkc_options *opt, void *stream,
                           ebbkc_graph **out);

/* Exact number of k-cliques: the k-vertex subsets of V whose vertices are
 * pairwise adjacent (the k-clique listing problem, Section 2).  k=1 gives n,
 * k=2 gives m (the l = 1 and l = 2 terminations of Algorithm EBBkC); k>=3
 * runs the edge-oriented branch and bound (Eq. edge-oriented-branching,
 * Section 4.1, every k-clique counted once under its first edge in pi_tau).
 * out_count: host pointer, written on EBBKC_OK.  Errors: EBBKC_E_K_RANGE for
 * k < 1 or k beyond the deepest search (278); EBBKC_E_OVERFLOW when the count
 * reaches 2^64 (ebbkc_count128 gives it); EBBKC_E_OOM / EBBKC_E_HIP. */
ebbkc_status ebbkc_count(ebbkc_graph *g, int32_t k, uint64_t *out_count, void *stream);

/* The same count as ebbkc_count, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): this call allocates nothing -- no hipMalloc, hipFree,
 * event or host allocation.  Its task lists, sort buffers and deep-search
 * frames live in a fixed per-device buffer of 256 MiB that the library holds
 * on every device it is loaded on until the process ends.  Every call on a device shares that device's
 * buffer: calls that overlap on one device race and must not be issued
 * concurrently (the buffer keeps the last call's contents; a call writes
 * everything it reads).
 *   g       a handle whose sub-branch arena exists (any earlier ebbkc_count at
 *           k >= 4, ebbkc_count_seeds or ebbkc_list builds it); otherwise
 *           EBBKC_E_INVALID_ARG.  The count always uses the edge roots and the
 *           colour-ordered search below them (the count is the same under every
 *           ebbkc_options.ordering).
 *   k       as for ebbkc_count (k = 1 gives n, k = 2 gives m).
 *   out_count  host pointer, written on EBBKC_OK.
 * Errors: EBBKC_E_SCRATCH when the count's task list (about 40 bytes per task
 * plus 12 bytes per seed) exceeds the fixed buffer; EBBKC_E_OVERFLOW past
 * 2^64; EBBKC_E_HIP when the buffer's address cannot be obtained. */
ebbkc_status ebbkc_count_noalloc(ebbkc_graph *g, int32_t k, uint64_t *out_count, void *stream);

/* The same count exactly in 128 bits: out_count[0] low word, out_count[1]
 * high word (near the maximum clique size counts pass 2^64: C(70, 35) > 2^64;
 * Section 6.2 (2) counts k up to omega).  E_OVERFLOW only past 2^128. */
ebbkc_status ebbkc_count128(ebbkc_graph *g, int32_t k, uint64_t out_count[2], void *stream);

/* Size omega of a maximum clique: the largest k with N_k > 0, by binary search
 * over k <= tau + 2 (Section 4.2: a seed's sub-branch has at most tau
 * vertices, so no clique exceeds tau + 2).  0 for an empty graph, 1 without
 * edges. */
ebbkc_status ebbkc_max_clique_size(ebbkc_graph *g, int32_t *out, void *stream);

/* Number of k-cliques whose seed edge (the edge of the clique that comes
 * first in the initial branch's edge order, pi_tau by default) has rank in
 * [r_begin, r_end).  Summed over a partition of
 * [0, m) this is the full count (every k-clique is listed exactly once,
 * Section 4.1).  k >= 3. */
ebbkc_status ebbkc_count_range(ebbkc_graph *g, int32_t k, int64_t r_begin, int64_t r_end,
                               uint64_t *out_count, void *stream);

/* Per-seed counts for the listed edge ids (device or host arrays per
 * ptr_kind): out[i] = number of k-cliques seeded by edge eids[i]. k >= 3. */
ebbkc_status ebbkc_count_seeds(ebbkc_graph *g, int32_t k, const int64_t *eids, int64_t ne,
                               int32_t ptr_kind, uint64_t *out, void *stream);

/* The k-cliques themselves (the listing of Section 2's problem; Algorithm
 * EBBkC outputs S plus each vertex (l = 1) or edge (l = 2) of the last
 * sub-branch, Algorithm kC2Plex the combinations of a 2-plex).
 * Write every k-clique (k >= 1) whose seed rank is in [r_begin, r_end) to
 * d_buf (device memory, cap tuples of k int32, row-major), each tuple in
 * ascending vertex order.  With EBBKC_LIST_SORTED the tuples are sorted
 * lexicographically.  *out_written is the number of tuples; if it exceeds
 * cap the call returns EBBKC_E_BUFFER_TOO_SMALL, sets *out_written to the
 * count and writes nothing else.  out_checksums (may be NULL) receives
 * [ordered, unordered]: with sm the SplitMix64 output function and h the
 * fold h <- sm(h ^ t_j) over the tuple from h = k, the unordered checksum is
 * sum_i h_i and the ordered one sum_i sm(h_i ^ sm(i)) over buffer positions
 * i (both mod 2^64; the ordered one is meaningful with SORTED).  Pass
 * r_begin = 0, r_end = -1 for the whole graph. */
ebbkc_status ebbkc_list(ebbkc_graph *g, int32_t k, int64_t r_begin, int64_t r_end, int32_t *d_buf,
                        uint64_t cap, uint32_t flags, uint64_t *out_written,
                        uint64_t *out_checksums, void *stream);

/* Copy one array (EBBKC_ARR_*) into dst (int32[m] for the per-edge arrays,
 * int32[n] for the per-vertex ones; host or device per ptr_kind).  A
 * per-vertex array the handle's ordering does not hold: EBBKC_E_INVALID_ARG. */
ebbkc_status ebbkc_export(const ebbkc_graph *g, int32_t which, int32_t *dst, int32_t ptr_kind,
                          void *stream);

ebbkc_status ebbkc_info_get(const ebbkc_graph *g, ebbkc_info *out);

/* Device time in milliseconds of the branch-kernel launch of each bitmap
 * width class in the last count call: out_ms[W-1] for sub-branches of at
 * most 64*W vertices (0 when that class was not launched), measured with HIP
 * events on the call's stream. */
ebbkc_status ebbkc_last_timing(const ebbkc_graph *g, double out_ms[4]);

/* Search work of the last count call, filled only when the handle was
 * prepared with ebbkc_options.count_work = 1 (otherwise zeros):
 * [0] seeds whose sub-branch was built, [1] search nodes evaluated,
 * [2] 64-bit word operations on candidate bitmaps (one AND + popcount of
 * one word each), [3] search nodes handed to another wave through the split
 * queue (node_split). */
ebbkc_status ebbkc_last_work(const ebbkc_graph *g, uint64_t out[4]);

/* The same counters for the launch of one bitmap width class
 * (width_class = W in 1..4: sub-branches of at most 64*W vertices), so that
 * a launch's work can be set against its time from ebbkc_last_timing; out[3]
 * is that launch's wave-finish tail in nanoseconds (its last wave's end minus
 * the mean end of its waves).
 * E_INVALID_ARG for a class outside 1..4. */
ebbkc_status ebbkc_last_work_class(const ebbkc_graph *g, int32_t width_class, uint64_t out[4]);

void ebbkc_destroy(ebbkc_graph *g);

/* ---- Batched form: many (graph, k) counts in one fused launch.
 * The tasks of every graph of the batch (one per seed sub-branch with at
 * least k-2 vertices; heavy roots split per first vertex) are merged into one
 * list sorted by bitmap width and by the vertices each task can still use,
 * and run by one persistent launch per width class, so the waves draw work
 * from all graphs at once (root sub-branches are independent, Section 6.2
 * (7)).  Counts are exact per graph. */
typedef struct ebbkc_batch ebbkc_batch;

/* graphs: n prepared handles on the current device (they must outlive the
 * batch and must not be used concurrently); ks: k per graph (k >= 1).  Builds
 * any missing sub-branch arenas and the merged task list.  opt may be NULL:
 * then a tuning choice cached for this batch shape is used if present. */
ebbkc_status ebbkc_batch_create(ebbkc_graph *const *graphs, const int32_t *ks, int32_t n,
                                const ebbkc_options *opt, void *stream, ebbkc_batch **out);

/* Run the batch and write the exact count of graph i to out_counts[i] (may be
 * NULL).  use_graph = 1 replays a HIP graph captured on the first call (the
 * counter reset, the per-class launches and the result copy); 0 launches the
 * same sequence directly.  Synchronises stream.  A failure belongs to the
 * graph that met it: a graph whose count reaches 2^64 gets 0 in out_counts
 * and the call returns EBBKC_E_OVERFLOW, while every other graph's count is
 * still written (out_counts is written in full whenever the launches ran). */
ebbkc_status ebbkc_batch_run(ebbkc_batch *b, int32_t use_graph, uint64_t *out_counts, void *stream);

/* Autotuner: times the batch under split thresholds {2^16, 2^22, 2^28, never}
 * (only the current one when the batch's tasks build their sub-branches, one
 * task per seed) x workgroups per CU {auto, 1, 2, not persistent}, then, with
 * the fastest of those, the runtime node split bounds {off, 2^10, 2^16, 2^22}
 * (ebbkc_options.node_split: how small a node may still be handed to an idle
 * wave, i.e. how deep a branch is spread over waves); checks every setting
 * gives the same counts and keeps the fastest (also in the process cache and,
 * if the environment names one, the EBBKC_TUNE_CACHE file).  Any out pointer
 * may be NULL. */
ebbkc_status ebbkc_batch_tune(ebbkc_batch *b, void *stream, int32_t *out_split, int32_t *out_blocks_per_cu,
                              int32_t *out_node_split);

/* Number of tasks and the host wall time (ms) of the last run. */
ebbkc_status ebbkc_batch_info(const ebbkc_batch *b, int64_t *out_tasks, double *out_last_ms);

void ebbkc_batch_destroy(ebbkc_batch *b);

/* ---- Served form: continuous batching of count requests.
 * A catalogue of prepared graphs stays resident in device memory; requests
 * (graph index, k) are submitted as they arrive.  A worker thread keeps up to
 * three epochs in flight, each on its own stream: an epoch takes the waiting
 * requests in arrival order while the estimated footprint of all epochs in
 * flight fits budget_bytes (a request larger than the budget runs when
 * nothing else does) and counts them in one fused batched launch per width
 * class.  Each launch leaves one workgroup slot per compute unit free, so
 * requests arriving while a long epoch runs start at once in another slot.  Results are exact and do not depend on which requests share an
 * epoch.  Times are milliseconds since the server was created (host steady
 * clock). */
typedef struct ebbkc_server ebbkc_server;

typedef struct {
    int64_t id;
    int32_t graph, k;
    int32_t status;     /* ebbkc_status of the request */
    int32_t pad;
    uint64_t count;     /* exact k-clique count (valid when status == EBBKC_OK) */
    double arrival_ms;  /* submission */
    double admit_ms;    /* start of the epoch that ran it */
    double done_ms;     /* result available */
} ebbkc_result;

/* graphs: the catalogue of n prepared handles on the current device (they
 * must outlive the server and not be used elsewhere while it runs); opt as
 * for ebbkc_batch_create (NULL: defaults).  budget_bytes > 0 bounds the
 * estimated device footprint of one epoch: per request 16 bytes per seed task
 * plus, for each of the 4096 waves a persistent launch can keep resident, one
 * bitmap of (tau+2)^2 bits (a sub-branch has at most tau vertices, Section
 * 4.2).  Builds the sub-branch arenas up front and starts the worker thread.
 * E_INVALID_ARG for a NULL handle, n <= 0 or budget_bytes <= 0; E_OOM / E_HIP
 * when an arena or the stream cannot be created.  The counts are the
 * k-clique counts of Section 2, as ebbkc_count gives them. */
ebbkc_status ebbkc_server_create(ebbkc_graph *const *graphs, int32_t n, const ebbkc_options *opt,
                                 int64_t budget_bytes, ebbkc_server **out);
/* Queue a request for the count of k-cliques (k >= 1) of catalogue graph
 * `graph`; *out_id identifies its result.  Never blocks on the device.
 * E_INVALID_ARG for a graph index outside the catalogue or k < 1; E_K_RANGE
 * for a k beyond the deepest search the library runs (2 + 2 * 136 + 4 = 278).
 * Each request's result carries its own status: a request whose count
 * reaches 2^64 reports EBBKC_E_OVERFLOW while the requests that shared its
 * epoch keep their counts, and an epoch of several requests that cannot start
 * (device memory, a runtime error) is retried one request per epoch. */
ebbkc_status ebbkc_server_submit(ebbkc_server *s, int32_t graph, int32_t k, int64_t *out_id);
/* Withdraw request id.  A request still waiting is removed at once and its
 * result (status EBBKC_E_CANCELLED, count 0) is available to poll; a request
 * whose epoch is already running finishes with that epoch but reports
 * EBBKC_E_CANCELLED.  E_INVALID_ARG for an unknown id or one whose result is
 * already available. */
ebbkc_status ebbkc_server_cancel(ebbkc_server *s, int64_t id);
/* Move up to max completed results to out (*n_out of them, in completion
 * order; the caller owns out, max entries); wait = 1 blocks until at least
 * one is available or nothing is pending.  A failed request is a result with
 * its status set and count 0. */
ebbkc_status ebbkc_server_poll(ebbkc_server *s, ebbkc_result *out, int32_t max, int32_t wait, int32_t *n_out);
/* [requests submitted, epochs run, most requests in one epoch, requests waiting or running] */
ebbkc_status ebbkc_server_stats(const ebbkc_server *s, int64_t out[4]);
/* Finishes the requests already submitted, stops the worker and frees the
 * server (not the catalogue's handles). */
void ebbkc_server_destroy(ebbkc_server *s);

const char *ebbkc_strerror(ebbkc_status s);

#ifdef __cplusplus
}
#endif
#endif /* EBBKC_H */
