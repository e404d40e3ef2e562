// arena.h -- the sub-branch arena: every seed's g_i built once per graph and
// kept in HBM (bitmap rows in colour order, colours, global vertex ids), and
// the task lists the search kernels pull from.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebb {

enum : int { ERR_WIDTH = 1, ERR_OVERFLOW = 2, ERR_DEPTH = 4, ERR_CAP = 8, ERR_QUEUE = 16 };
enum : int { OPT_ET = 1, OPT_RULE1 = 4, OPT_RULE2 = 8, OPT_WORK = 16 };

constexpr int MAX_W = 4;                 // widest bitmap class: 256 vertices
constexpr int ADJ_DEFAULT_MAX_N = 8192;  // graphs up to this many vertices get an adjacency bitmap
constexpr int ADJ_MAX_N = 32768;         // largest bound the option accepts (128 MB bitmap)
constexpr int LIST_FUSED_K = 8;          // listings up to this k sort and hash tuples as they are written
constexpr int LDS_FRAMES = 12;           // search frames kept in LDS (nodes with l >= 6)
constexpr int GLOBAL_FRAMES = 124;       // further frames in device memory, per wave
constexpr int LIST_LDS_FRAMES = 16;      // listing frames kept in LDS
// a search at k needs device-memory frames past these k (count kernel,
// listing kernel); a listing runs both kernels
constexpr int SEARCH_DEEP_K = 2 + 2 * LDS_FRAMES + 4;
constexpr int LIST_DEEP_K = 2 + 2 * LIST_LDS_FRAMES + 2;
constexpr int MAX_K = 2 + 2 * (LDS_FRAMES + GLOBAL_FRAMES) + 4;

// Graph arrays the build kernel reads.
struct GraphView {
    const int32_t* rp;
    const int32_t* ci;
    const int32_t* erank;
    const int2* rrow;
    const int32_t* orp;
    const int2* orow;
    const int32_t* eu;
    const int32_t* ev;
    const int32_t* rank;
    // adjacency bitmap of G (graphs of at most a few thousand vertices; null
    // otherwise): row x holds adjw words, bit w set for every neighbour w;
    // acum[x adjw + q] = entries of x's id-sorted row below vertex 64 q
    const uint64_t* adj;
    const uint16_t* acum;
    int32_t adjw;
};

// Seeds are the edges with |V(g_i)| >= 1 in rank order; slot s of the arena
// holds seed s.
struct ArenaView {
    const int32_t* seed_eid;  // edge id of slot s
    const int32_t* seed_c;    // |V(g_i)| of slot s
    const int64_t* row_off;   // first 64-bit word of slot s's rows (c * W words)
    const int64_t* vtx_off;   // first vertex entry of slot s (c entries)
    const uint64_t* rows;     // symmetric adjacency rows, vertices in colour order
    const int32_t* gid;       // global id of each local vertex
    const int16_t* col;       // colour of each local vertex (non-increasing)
};

struct BuildArgs {
    GraphView G;
    const int32_t* list;  // slots to build (one width class)
    int64_t n;
    const int32_t* seed_eid;
    const int32_t* seed_c;
    const int64_t* row_off;
    const int64_t* vtx_off;
    uint64_t* rows;
    int32_t* gid;
    int16_t* col;
    uint64_t* nedges;  // edges of g_i per slot
    const int32_t* vcol;  // colours of G kept in every g_i, or null: each g_i coloured on its own
    const int32_t* seed_rthr;  // vertex slots: seed_eid holds the vertex, its sub-branch is its
                               // neighbourhood through edges ranked after seed_rthr; null: edge slots
    unsigned long long* next;
    int* err;
};

// task = slot << 20 | x0 << 10 | x1 : the children of the root whose first
// vertex x lies in [x0, x1)
__host__ __device__ inline int64_t task_pack(int64_t slot, int x0, int x1) {
    return (slot << 20) | ((int64_t)x0 << 10) | (int64_t)x1;
}
__host__ __device__ inline int64_t task_slot(int64_t t) { return t >> 20; }
__host__ __device__ inline int task_x0(int64_t t) { return (int)((t >> 10) & 1023); }
__host__ __device__ inline int task_x1(int64_t t) { return (int)(t & 1023); }

// The root tasks of a slot with c vertices at l0 = k-2 (needs c >= l0): one
// task [0, c) unless the root's work bound log C(c, l0) exceeds the split
// threshold; then ranges [x0, x1) of first root vertices.  Root vertex x heads
// at most C(c-1-x, l0-1) cliques; consecutive vertices are grouped until their
// bound reaches that of x = 0, so no task is heavier than the heaviest single
// vertex and light vertices do not each reload the slot.  Calls emit(x0, x1)
// for every task and returns their number.
__device__ inline double log_binom(int n, int r) {
    return lgamma((double)n + 1) - lgamma((double)r + 1) - lgamma((double)(n - r) + 1);
}
template <class F>
__device__ inline int root_tasks(int c, int l0, double log_threshold, F&& emit) {
    if (l0 < 4 || c < l0 + 8 || log_binom(c, l0) <= log_threshold) {
        emit(0, c);
        return 1;
    }
    const double top = log_binom(c - 1, l0 - 1);
    const int last = c - l0;
    int n = 0, x0 = 0;
    double acc = 0.0;
    for (int x = 0; x <= last; ++x) {
        acc += exp(log_binom(c - 1 - x, l0 - 1) - top);
        if (acc >= 0.999 || x == last) {
            emit(x0, x + 1);
            ++n;
            x0 = x + 1;
            acc = 0.0;
        }
    }
    return n;
}

// Runtime splitting: a search node handed from one wave to any idle wave
// through a device queue (root sub-branches and their subtrees are
// independent, Section 6.2 (7)).  The item names the task it came from
// (which gives the slot, graph and k), the node's candidate set and l.
struct SplitItem {
    int64_t it;
    uint64_t P[MAX_W];
    int32_t l;
    int32_t ready;  // 1 once the item is written (release store)
};
// queue counters, each on a 128-byte line of its own (waiting waves poll
// them while working waves update them): [SQ_HEAD] items claimed,
// [SQ_RESERVE] items reserved, [SQ_BUSY] waves working (a wave counts itself
// when it starts), [SQ_IDLE] waves waiting for items, [SQ_PUSHED] items
// pushed over the launch
enum : int { SQ_HEAD = 0, SQ_RESERVE = 16, SQ_BUSY = 32, SQ_IDLE = 48, SQ_PUSHED = 64, SQ_WORDS = 80 };
constexpr int64_t SQ_CAP = 1 << 16;        // items per launch
constexpr int64_t SQ_SLACK = 1 << 13;       // more than the waves of one launch
constexpr int SPLIT_OFF = 0, SPLIT_ON_DEMAND = 1, SPLIT_FORCED = 2;
// default bound of runtime splitting: a node is handed over only if it has at
// least this many l-subsets (2^16 pushed so many small nodes that the queue
// filled early and its round trips cost more than they saved; 2^20 was best
// on R-MAT s12/s13 and Chung-Lu 3e5 at k = 11, 12)
constexpr uint64_t NODE_SPLIT_DEFAULT = 1ull << 20;

// A graph whose sub-branches are built by the search tasks themselves (no
// arena): its arrays, |V(g_i)| of every edge, and the colours of G kept in
// every g_i under EBBkC-C (null: each g_i coloured on its own).
struct BuildGraph {
    GraphView G;
    const int32_t* subsize;
    const int32_t* vcol;
};
struct SearchArgs {
    ArenaView A;
    const int64_t* tasks;
    int64_t ntasks;
    int32_t k;
    int32_t opts;
    float k4_weight;            // dense 4-clique evaluation cost weight (<= 0: never)
    int32_t tplex;              // largest t counted in closed form (1..3), 0: 2 when 2k <= tau, else 3
    int32_t tau;                // the graph's tau (for tplex = 0)
    unsigned long long* next;
    unsigned long long* total;  // [lo, hi]
    unsigned long long* work;   // [tasks, nodes, word ops]
    int* err;
    uint64_t* per_task;         // optional count per task (indexed like tasks)
    void* gframes;              // GLOBAL_FRAMES frames per wave of the grid
    // listing (per_task offsets of the output, tuples of k int32)
    const uint64_t* task_off;
    int32_t* out;
    const int32_t* eu;
    const int32_t* ev;
    // k <= 8: tuples written sorted and hashed as they are emitted, checksums
    // [ordered, unordered] added here (null: written as found, sorted later)
    unsigned long long* list_checksums;
    // batches of graphs: task i belongs to graph task_graph[i], whose arena is
    // views[g] and whose clique size is graph_k[g]; its count is added to
    // graph_total[2g] (low word) / [2g+1] (high word)
    const ArenaView* views;
    const int32_t* task_graph;
    const int32_t* graph_k;
    const int32_t* graph_tau;
    unsigned long long* graph_total;
    // batches whose tasks build their own sub-branch (the search kernel's
    // build variant): graph g's arrays; a task's slot is its seed edge id
    const BuildGraph* bviews;
    // runtime splitting (squeue null: off).  SPLIT_ON_DEMAND: a node with
    // l >= 4 whose bound C(|P|, l) reaches split_bound is pushed while waves
    // wait for work and fewer items are pending than waves wait; SPLIT_FORCED:
    // every such node is pushed while the queue has room (a test of the
    // queue at every depth)
    SplitItem* squeue;
    unsigned long long* sq;      // SQ_WORDS counters, zeroed before the launch
    int32_t split_mode;
    uint64_t split_bound;
    // when counting work: [sum of wave end times, latest end, waves, ~earliest
    // start] in 10 ns ticks of the constant-rate clock
    unsigned long long* wave_time;
};

// EBBkC-T search (one launch per width class): the fields mean what they mean
// in SearchArgs; rp / ci / erank are the graph's CSR with edge ranks, rho a
// slab of truss_slab_bytes(cus) bytes (a c x c rank matrix per wave)
constexpr int TRUSS_FRAMES = 48;        // branching depth: k <= 2 * TRUSS_FRAMES + 3
constexpr int TRUSS_BLOCKS_PER_CU = 4;   // three fit at W = 4 (LDS); a fourth finds the queue empty
struct TrussArgs {
    ArenaView A;
    const int64_t* tasks;
    int64_t ntasks;
    int32_t k;
    int32_t opts;
    int32_t tplex;
    const int32_t* rp;
    const int32_t* ci;
    const int32_t* erank;
    int32_t* rho;
    unsigned long long* next;
    unsigned long long* total;
    unsigned long long* work;
    int* err;
    uint64_t* per_task;
};

hipError_t launch_build(int W, const BuildArgs& a, int cus, hipStream_t s);
hipError_t launch_search_truss(int W, const TrussArgs& a, int cus, hipStream_t s);
size_t truss_slab_bytes(int cus);
hipError_t launch_search(int W, bool build, const SearchArgs& a, int cus, int blocks_per_cu, hipStream_t s);
int64_t search_grid_waves(int W, bool build, int64_t ntasks, int cus, int blocks_per_cu);
size_t search_frame_bytes(int W);
hipError_t launch_binom_init(hipStream_t s);
hipError_t launch_sq_reset(unsigned long long* sq, SplitItem* items, hipStream_t s);
float k4_weight_of(int32_t dense_k4);
hipError_t launch_list(int W, const SearchArgs& a, int cus, hipStream_t s);
size_t list_frame_bytes(int W);
int64_t list_grid_waves(int W, int64_t ntasks, int cus);
hipError_t canon_tuples(int32_t* buf, int64_t n, int k, hipStream_t s);
hipError_t sort_tuples(int32_t* buf, int64_t n, int k, int bits, uint64_t* keys, uint64_t* keys2, uint32_t* idx,
                       uint32_t* idx2, int64_t* hist, int64_t* htmp, int32_t* tmpbuf, hipStream_t s);
hipError_t tuple_checksums(const int32_t* buf, int64_t n, int k, unsigned long long* d_out, hipStream_t s);
hipError_t list_small(const int32_t* byrank, const int32_t* eu, const int32_t* ev, int64_t lo, int64_t hi, int k,
                      int32_t* out, hipStream_t s);
hipError_t launch_subsize(const GraphView& G, int64_t m, int32_t* out, hipStream_t s);

}  // namespace ebb
