// batch.hip -- many (graph, k) counts in one fused launch per bitmap width
// class, captured once in a HIP graph and replayed.
//
// Every graph of the batch is prepared; its sub-branches come from its arena
// or, for batches whose arenas would not fit device memory, are built by
// each task in LDS.  The tasks of all graphs (as in a single count: one per
// seed with enough vertices, heavy roots split per first vertex when the
// sub-branches come from arenas) are merged into one list, sorted by width
// class and then by the vertices a task can still use, largest first (tasks
// that build: by graph first, so a launch works on one graph's arrays at a
// time), so the persistent waves of one launch draw work from every graph.
// Each task adds its count to its own graph's exact 128-bit total; a served
// epoch is such a batch, without runtime node splitting.
//
// Autotuning: ebbkc_batch_tune times the batch under a few (split threshold,
// workgroups per CU) settings, then, with the best of those, a few bounds for
// handing search nodes to idle waves at run time (how deep a branch is split
// over waves), and keeps the fastest; the choice is cached per batch
// signature for the process (and in the file named by EBBKC_TUNE_CACHE when
// that variable is set).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "arena.h"
#include "common.h"
#include "handle.h"
#include "prims.h"

struct ebbkc_batch {
    int device = 0;
    std::vector<ebbkc_graph*> graphs;
    std::vector<int32_t> ks;
    ebbkc_options opt{};
    int cu_count = 256;
    // sub-branches: loaded from every graph's arena, or built by each task in
    // LDS from the graph's arrays (bviews)
    bool build = false;
    ebb::BuildGraph* bviews = nullptr;
    // device
    ebb::ArenaView* views = nullptr;
    int32_t* gk = nullptr;
    int32_t* gtau = nullptr;
    int64_t* tasks = nullptr;
    int32_t* tgraph = nullptr;
    unsigned long long* gtot = nullptr;  // 2 per graph
    unsigned long long* ctr = nullptr;   // [0..4) class work counters, [4..6) unused, [6] err, [8..11] work
    ebb::SplitItem* squeue = nullptr;    // runtime split queue (null: off)
    unsigned long long* sq = nullptr;
    void* gframes = nullptr;
    int64_t ntasks = 0;
    uint64_t ccount[4] = {0, 0, 0, 0};
    int32_t kmax = 0;
    // host results
    unsigned long long* h_tot = nullptr;
    unsigned long long* h_ctr = nullptr;
    // captured launch sequence
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool dirty = true;  // tasks changed since capture
    double last_ms = 0.0;
    // device memory: stream-ordered on mem_stream when async_mem (the served
    // form, whose epochs overlap: a plain free would wait for the device)
    bool async_mem = false;
    hipStream_t mem_stream = nullptr;
    bool own_host = true;  // h_tot / h_ctr allocated by the batch
};

namespace ebb {
namespace {

#define CHKB(expr)                                                              \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) {                                                 \
            (void)hipGetLastError();                                            \
            return e_ == hipErrorOutOfMemory ? EBBKC_E_OOM : EBBKC_E_HIP;       \
        }                                                                       \
    } while (0)

__host__ __device__ inline int width_of(int c) { return c <= 64 ? 1 : (c <= 128 ? 2 : (c <= 192 ? 3 : 4)); }

inline unsigned gridn(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (unsigned)b;
}

__global__ void k_btask_counts(const int32_t* __restrict__ seed_c, int64_t n, int l0, double log_thr,
                               int32_t* __restrict__ tcount) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = seed_c[i];
        tcount[i] = c >= l0 ? root_tasks(c, l0, log_thr, [](int, int) {}) : 0;
    }
}

// Sort key of a task: width class, then (gbits > 0) its graph, then the
// vertices it can still use, largest first.
__global__ void k_btask_fill(const int32_t* __restrict__ seed_c, int64_t n, int l0, double log_thr,
                             const int64_t* __restrict__ toff, int64_t base, int32_t graph, int gbits,
                             int64_t* __restrict__ tasks, int32_t* __restrict__ tgraph, uint64_t* __restrict__ keys,
                             uint32_t* __restrict__ vals) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = seed_c[i];
        if (c < l0) continue;
        const int W = width_of(c);
        int64_t o = base + toff[i];
        root_tasks(c, l0, log_thr, [&](int x0, int x1) {
            tasks[o] = task_pack(i, x0, x1);
            tgraph[o] = graph;
            const int usable = x0 == 0 && x1 >= c ? c : c - 1 - x0;
            keys[o] = ((uint64_t)(W - 1) << (8 + gbits)) | ((uint64_t)(gbits ? graph : 0) << 8) |
                      (uint64_t)(255 - (usable > 255 ? 255 : usable));
            vals[o] = (uint32_t)o;
            ++o;
        });
    }
}

__global__ void k_bgather(const int64_t* __restrict__ tasks, const int32_t* __restrict__ tgraph,
                          const uint32_t* __restrict__ idx, int64_t n, int64_t* __restrict__ otasks,
                          int32_t* __restrict__ ograph) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        otasks[i] = tasks[idx[i]];
        ograph[i] = tgraph[idx[i]];
    }
}

// tasks per width class: counted per lane, summed per wave, one atomic per
// wave and class (one atomic per task on four counters took 17 s for the
// 1.46e9 tasks of the 4,096-graph batch)
__global__ void k_bclass_hist(const uint64_t* __restrict__ keys, int64_t n, int gbits,
                              unsigned long long* __restrict__ cls) {
    uint64_t per_class[4] = {0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int w = (int)((keys[i] >> (8 + gbits)) & 3);
#pragma unroll
        for (int q = 0; q < 4; ++q) per_class[q] += q == w ? 1 : 0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t t = wave_sum(per_class[q]);
        if (lane_id() == 0 && t) atomicAdd(&cls[q], (unsigned long long)t);
    }
}

// zero the counters and per-graph totals (a kernel, so the captured graph
// holds no memset node)
__global__ void k_bclear(unsigned long long* __restrict__ a, int64_t na, unsigned long long* __restrict__ b,
                         int64_t nb) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < na) a[i] = 0;
        else b[i - na] = 0;
    }
}

// bytes of the arena slots of graph g (|V(g_i)| >= 1): c W words of rows plus
// 6 bytes of id and colour per vertex; and the widest sub-branch
__global__ void k_arena_bytes(const int32_t* __restrict__ subsize, int64_t m, unsigned long long* __restrict__ out) {
    uint64_t b = 0;
    int mx = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = subsize[e];
        if (c > 0) b += (uint64_t)c * (uint64_t)width_of(c) * 8 + 6 * (uint64_t)c;
        mx = c > mx ? c : mx;
    }
    b = wave_sum(b);
    mx = wave_max(mx);
    if (lane_id() == 0) {
        if (b) atomicAdd(&out[0], (unsigned long long)b);
        atomicMax(&out[1], (unsigned long long)mx);
    }
}

GraphView graph_arrays(const ebbkc_graph* g) {
    return GraphView{g->rp, g->ci, g->erank, g->rrow, g->orp, g->orow, g->eu, g->ev, g->rank,
                     g->adj, g->acum, g->adjw};
}

int opts_of(const ebbkc_options& o) {
    int f = 0;
    if (o.early_termination) f |= OPT_ET;
    if (o.rule1) f |= OPT_RULE1;
    if (o.rule2) f |= OPT_RULE2;
    return f;
}

hipError_t dev_alloc(const ebbkc_batch* b, void** p, size_t bytes, hipStream_t s) {
    return b->async_mem ? hipMallocAsync(p, bytes, s) : hipMalloc(p, bytes);
}
void dev_free(const ebbkc_batch* b, void* p, hipStream_t s) {
    if (!p) return;
    if (b->async_mem) (void)hipFreeAsync(p, s);
    else (void)hipFree(p);
}

void free_tasks(ebbkc_batch* b) {
    dev_free(b, b->tasks, b->mem_stream);
    dev_free(b, b->tgraph, b->mem_stream);
    dev_free(b, b->gframes, b->mem_stream);
    b->tasks = nullptr;
    b->tgraph = nullptr;
    b->gframes = nullptr;
    b->ntasks = 0;
    b->dirty = true;
}

// Build the merged, sorted task list under the batch's current options.
ebbkc_status build_tasks(ebbkc_batch* b, hipStream_t s) {
    free_tasks(b);
    const int n = (int)b->graphs.size();
    const double thr = b->opt.split_threshold > 0 ? (double)b->opt.split_threshold : (double)(1 << 22);
    // a task that builds its g_i would rebuild it for every root range: one
    // task per seed there (the runtime split queue balances heavy ones)
    const double log_thr = b->opt.split_threshold < 0 || b->build ? 1e300 : std::log(thr);
    // per graph: task counts and offsets (scratch sized for the largest graph)
    std::vector<int64_t> gbase((size_t)n + 1, 0);
    std::vector<int64_t*> toffs((size_t)n, nullptr);
    // seeds: arena slots, or (build mode) every edge with its |V(g_i)|
    auto seeds_of = [&](const ebbkc_graph* g) -> int64_t { return b->build ? g->m : g->nseeds; };
    auto sizes_of = [&](const ebbkc_graph* g) -> const int32_t* { return b->build ? g->subsize : g->seed_c; };
    int64_t total = 0, nsmax = 0;
    for (int i = 0; i < n; ++i) nsmax = std::max(nsmax, seeds_of(b->graphs[(size_t)i]));
    int32_t* tc = nullptr;
    int64_t* tmp = nullptr;
    CHKB(dev_alloc(b, (void**)&tc, sizeof(int32_t) * (nsmax + 1), s));
    CHKB(dev_alloc(b, (void**)&tmp, sizeof(int64_t) * (scan_tmp_elems(nsmax + 1) + 64), s));
    std::vector<int64_t> tcount((size_t)n, 0);
    for (int i = 0; i < n; ++i) {
        ebbkc_graph* g = b->graphs[(size_t)i];
        const int k = b->ks[(size_t)i];
        if (k < 3 || seeds_of(g) == 0) continue;
        const int64_t ns = seeds_of(g);
        int64_t* to = nullptr;
        CHKB(dev_alloc(b, (void**)&to, sizeof(int64_t) * (ns + 1), s));
        hipLaunchKernelGGL(k_btask_counts, dim3(gridn(ns)), dim3(256), 0, s, sizes_of(g), ns, k - 2, log_thr, tc);
        CHKB(exclusive_scan_i32(tc, to, ns, to + ns, tmp, s));
        CHKB(hipMemcpyAsync(&tcount[(size_t)i], to + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        toffs[(size_t)i] = to;
    }
    CHKB(hipStreamSynchronize(s));
    dev_free(b, tc, s);
    dev_free(b, tmp, s);
    for (int i = 0; i < n; ++i) {
        gbase[(size_t)i] = total;
        total += tcount[(size_t)i];
    }
    gbase[(size_t)n] = total;
    b->ntasks = total;
    if (total == 0) {
        for (auto p : toffs) dev_free(b, p, s);
        return EBBKC_OK;
    }
    if (total >= ((int64_t)1 << 32)) return EBBKC_E_OOM;
    int64_t *tasks = nullptr, *hist = nullptr, *htmp = nullptr;
    int32_t* tg = nullptr;
    uint64_t *keys = nullptr, *keys2 = nullptr;
    uint32_t *vals = nullptr, *vals2 = nullptr;
    const int64_t hn = radix_hist_elems(total);
    CHKB(dev_alloc(b, (void**)&tasks, sizeof(int64_t) * total, s));
    CHKB(dev_alloc(b, (void**)&tg, sizeof(int32_t) * total, s));
    CHKB(dev_alloc(b, (void**)&keys, sizeof(uint64_t) * total, s));
    CHKB(dev_alloc(b, (void**)&keys2, sizeof(uint64_t) * total, s));
    CHKB(dev_alloc(b, (void**)&vals, sizeof(uint32_t) * total, s));
    CHKB(dev_alloc(b, (void**)&vals2, sizeof(uint32_t) * total, s));
    CHKB(dev_alloc(b, (void**)&hist, sizeof(int64_t) * hn, s));
    CHKB(dev_alloc(b, (void**)&htmp, sizeof(int64_t) * (scan_tmp_elems(hn) + 64), s));
    // tasks that build their g_i run graph by graph within a width class, so
    // that the waves of a launch share one graph's arrays in cache
    int gbits = 0;
    if (b->build)
        while (((int64_t)1 << gbits) < (int64_t)n) ++gbits;
    for (int i = 0; i < n; ++i) {
        if (!toffs[(size_t)i]) continue;
        ebbkc_graph* g = b->graphs[(size_t)i];
        hipLaunchKernelGGL(k_btask_fill, dim3(gridn(seeds_of(g))), dim3(256), 0, s, sizes_of(g), seeds_of(g),
                           b->ks[(size_t)i] - 2, log_thr, toffs[(size_t)i], gbase[(size_t)i], (int32_t)i, gbits, tasks,
                           tg, keys, vals);
    }
    CHKB(radix_sort_u64(keys, vals, keys2, vals2, total, 10 + gbits, hist, htmp, s));
    CHKB(dev_alloc(b, (void**)&b->tasks, sizeof(int64_t) * total, s));
    CHKB(dev_alloc(b, (void**)&b->tgraph, sizeof(int32_t) * total, s));
    hipLaunchKernelGGL(k_bgather, dim3(gridn(total)), dim3(256), 0, s, tasks, tg, vals, total, b->tasks, b->tgraph);
    CHKB(hipMemsetAsync(b->ctr, 0, 16 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_bclass_hist, dim3(gridn(total)), dim3(256), 0, s, keys, total, gbits, b->ctr);
    unsigned long long cc[4];
    CHKB(hipMemcpyAsync(cc, b->ctr, sizeof(cc), hipMemcpyDeviceToHost, s));
    CHKB(hipStreamSynchronize(s));
    for (int w = 0; w < 4; ++w) b->ccount[w] = cc[w];
    for (auto p : toffs) dev_free(b, p, s);
    void* ptrs[] = {tasks, tg, keys, keys2, vals, vals2, hist, htmp};
    for (void* p : ptrs) dev_free(b, p, s);
    // frames for deep searches
    if (b->kmax > SEARCH_DEEP_K) {
        int64_t waves = 0;
        for (int W = 1; W <= MAX_W; ++W)
            waves = std::max(waves, search_grid_waves(W, b->build, total, b->cu_count, b->opt.blocks_per_cu));
        CHKB(dev_alloc(b, &b->gframes, (size_t)waves * GLOBAL_FRAMES * search_frame_bytes(MAX_W), s));
    }
    b->dirty = true;
    return EBBKC_OK;
}

// The launch sequence: clear counters, one search per width class, copy the
// per-graph totals and error flags to pinned host memory.
ebbkc_status enqueue(ebbkc_batch* b, hipStream_t s) {
    const int n = (int)b->graphs.size();
    hipLaunchKernelGGL(k_bclear, dim3(gridn(16 + 2 * (int64_t)n)), dim3(256), 0, s, b->ctr, (int64_t)16, b->gtot,
                       2 * (int64_t)n);
    CHKB(hipGetLastError());
    int64_t off = 0;
    for (int W = 1; W <= MAX_W; ++W) {
        const int64_t nt = (int64_t)b->ccount[W - 1];
        if (!nt) continue;
        SearchArgs a{};
        a.tasks = b->tasks + off;
        a.task_graph = b->tgraph + off;
        a.ntasks = nt;
        a.views = b->build ? nullptr : b->views;
        a.bviews = b->build ? b->bviews : nullptr;
        a.graph_k = b->gk;
        a.graph_total = b->gtot;
        a.opts = opts_of(b->opt);
        a.k4_weight = k4_weight_of(b->opt.dense_k4);
        a.tplex = b->opt.t_plex;
        a.graph_tau = b->gtau;
        a.next = b->ctr + (W - 1);
        a.total = b->ctr + 4;
        a.work = b->ctr + 8;
        a.err = (int*)(b->ctr + 6);
        a.gframes = b->gframes;
        // persistent grids only; not in served epochs, which run concurrently
        // (waves waiting for split nodes would hold compute units that the
        // other epochs need)
        if (b->squeue && !b->async_mem && b->opt.node_split != -1 && b->opt.blocks_per_cu != -1) {
            a.squeue = b->squeue;
            a.sq = b->sq;
            a.split_mode = b->opt.node_split == 1 ? SPLIT_FORCED : SPLIT_ON_DEMAND;
            a.split_bound = b->opt.node_split == 1 ? 0 : (b->opt.node_split >= 2 ? (uint64_t)b->opt.node_split : NODE_SPLIT_DEFAULT);
            CHKB(launch_sq_reset(b->sq, b->squeue, s));
        }
        CHKB(launch_search(W, b->build, a, b->cu_count, b->opt.blocks_per_cu, s));
        off += nt;
    }
    CHKB(hipMemcpyAsync(b->h_tot, b->gtot, sizeof(unsigned long long) * 2 * n, hipMemcpyDeviceToHost, s));
    CHKB(hipMemcpyAsync(b->h_ctr, b->ctr, sizeof(unsigned long long) * 16, hipMemcpyDeviceToHost, s));
    return EBBKC_OK;
}

ebbkc_status capture(ebbkc_batch* b, hipStream_t s) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    // capture on a private stream (the null stream cannot be captured)
    hipStream_t cs;
    CHKB(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    ebbkc_status st = EBBKC_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) st = EBBKC_E_HIP;
    if (!st) st = enqueue(b, cs);
    hipGraph_t gr = nullptr;
    if (hipStreamEndCapture(cs, &gr) != hipSuccess && !st) st = EBBKC_E_HIP;
    if (!st && hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0) != hipSuccess) st = EBBKC_E_HIP;
    b->graph = gr;
    (void)hipStreamDestroy(cs);
    (void)s;
    if (!st) b->dirty = false;
    return st;
}

// Results of the last run: the count of graph i into out[i] and, when
// status is given, its own status into status[i] (an overflow or a depth
// limit belongs to the graph that met it).  Returns the first failing status,
// or EBBKC_OK.
ebbkc_status finish(ebbkc_batch* b, uint64_t* out, ebbkc_status* status = nullptr) {
    const int n = (int)b->graphs.size();
    const int err = (int)b->h_ctr[6];
    ebbkc_status first = EBBKC_OK;
    for (int i = 0; i < n; ++i) {
        const int k = b->ks[(size_t)i];
        ebbkc_graph* g = b->graphs[(size_t)i];
        uint64_t v = 0;
        ebbkc_status st = EBBKC_OK;
        if (err & ERR_WIDTH) st = EBBKC_E_WIDTH;
        else if (err & ERR_QUEUE) st = EBBKC_E_HIP;
        else if ((err & ERR_DEPTH) && k > SEARCH_DEEP_K) st = EBBKC_E_K_RANGE;
        else if (k == 1) v = (uint64_t)g->n;
        else if (k == 2) v = (uint64_t)g->m;
        else if (k - 2 > g->tau) v = 0;
        else if (b->h_tot[2 * i + 1] != 0 || (err & ERR_OVERFLOW)) st = EBBKC_E_OVERFLOW;
        else v = b->h_tot[2 * i];
        if (out) out[i] = st ? 0 : v;
        if (status) status[i] = st;
        if (st && !first) first = st;
    }
    return first;
}

std::mutex g_tune_mu;
struct Tuned {
    int32_t split, bpc, node_split;
};
std::map<std::string, Tuned> g_tune_cache;

std::string signature(const ebbkc_batch* b) {
    // graphs, total seeds (log2 bucket), k histogram
    int64_t seeds = 0;
    int hist[16] = {0};
    for (size_t i = 0; i < b->graphs.size(); ++i) {
        seeds += b->graphs[i]->nseeds;
        hist[std::min(15, (int)b->ks[i])]++;
    }
    char buf[256];
    int o = snprintf(buf, sizeof(buf), "n%zu_s%d%s", b->graphs.size(), seeds > 0 ? (int)std::log2((double)seeds) : 0,
                     b->build ? "_build" : "");
    for (int k = 3; k < 16; ++k)
        if (hist[k]) o += snprintf(buf + o, sizeof(buf) - (size_t)o, "_k%d:%d", k, hist[k]);
    return std::string(buf);
}

void load_cache_file() {
    const char* path = getenv("EBBKC_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[256];
    int a, c, d;
    while (fscanf(f, "%255s %d %d %d", key, &a, &c, &d) == 4) g_tune_cache[key] = {a, c, d};
    fclose(f);
}

void save_cache_file() {
    const char* path = getenv("EBBKC_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "w");
    if (!f) return;
    for (auto& kv : g_tune_cache)
        fprintf(f, "%s %d %d %d\n", kv.first.c_str(), kv.second.split, kv.second.bpc, kv.second.node_split);
    fclose(f);
}

}  // namespace
}  // namespace ebb

namespace ebb {
namespace {

void batch_destroy_impl(ebbkc_batch* b) {
    if (!b) return;
    free_tasks(b);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void* ptrs[] = {b->views, b->bviews, b->gk, b->gtau, b->gtot, b->ctr, b->squeue, b->sq};
    for (void* p : ptrs) dev_free(b, p, b->mem_stream);
    if (b->own_host) {
        if (b->h_tot) (void)hipHostFree(b->h_tot);
        if (b->h_ctr) (void)hipHostFree(b->h_ctr);
    }
    delete b;
}

// Batch of n (graph, k) counts.  async_mem: device memory is stream-ordered on
// s; h_tot / h_ctr: caller-owned pinned result buffers (2 n and 16 words), or
// null to allocate them.  use_cache: take a cached tuning choice when opt is
// null.
ebbkc_status batch_create_impl(ebbkc_graph* const* graphs, const int32_t* ks, int32_t n, const ebbkc_options* opt,
                               hipStream_t s, bool async_mem, unsigned long long* h_tot, unsigned long long* h_ctr,
                               ebbkc_batch** out) {
    ebbkc_batch* b = new ebbkc_batch();
    b->async_mem = async_mem;
    b->mem_stream = s;
    b->graphs.assign(graphs, graphs + n);
    b->ks.assign(ks, ks + n);
    if (opt) b->opt = *opt; else ebbkc_default_options(&b->opt);
    b->opt.count_work = 0;
    (void)hipGetDevice(&b->device);
    if (hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
        delete b;
        return EBBKC_E_HIP;
    }
    std::vector<ArenaView> views((size_t)n);
    std::vector<BuildGraph> bviews((size_t)n);
    bool all_arenas = true;
    for (int i = 0; i < n; ++i) {
        ebbkc_graph* g = graphs[i];
        if (!g || g->device != b->device || ks[i] < 1 || ks[i] > MAX_K) { delete b; return EBBKC_E_INVALID_ARG; }
        b->kmax = std::max(b->kmax, ks[i]);
        if (ks[i] >= 3 && ks[i] - 2 <= g->tau && !g->arena_built) all_arenas = false;
    }
    // where the sub-branches come from: arenas, or built by each task in LDS
    // (auto: arenas when they exist already or fit half the free memory)
    int mode = b->opt.batch_build;
    if (mode == EBBKC_BATCH_AUTO && all_arenas) mode = EBBKC_BATCH_ARENA;
    if (mode != EBBKC_BATCH_ARENA) {
        unsigned long long* est = nullptr;
        if (hipMalloc((void**)&est, sizeof(unsigned long long) * 2 * n) != hipSuccess) { delete b; return EBBKC_E_OOM; }
        (void)hipMemsetAsync(est, 0, sizeof(unsigned long long) * 2 * n, s);
        for (int i = 0; i < n; ++i) {
            ebbkc_graph* g = graphs[i];
            if (ks[i] < 3 || ks[i] - 2 > g->tau) continue;
            ebbkc_status st = subsize_impl(g, s);
            if (st) { (void)hipFree(est); delete b; return st; }
            if (g->m) hipLaunchKernelGGL(k_arena_bytes, dim3(gridn(g->m)), dim3(256), 0, s, g->subsize, g->m, est + 2 * i);
        }
        std::vector<unsigned long long> h((size_t)2 * n);
        const bool ok = hipMemcpyAsync(h.data(), est, sizeof(unsigned long long) * 2 * n, hipMemcpyDeviceToHost, s) ==
                            hipSuccess && hipStreamSynchronize(s) == hipSuccess;
        (void)hipFree(est);
        if (!ok) { delete b; return EBBKC_E_HIP; }
        uint64_t need = 0, widest = 0;
        for (int i = 0; i < n; ++i) {
            if (!graphs[i]->arena_built) need += h[(size_t)2 * i];
            widest = std::max<uint64_t>(widest, h[(size_t)2 * i + 1]);
        }
        if (mode == EBBKC_BATCH_AUTO) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete b; return EBBKC_E_HIP; }
            mode = need <= fr / 2 ? EBBKC_BATCH_ARENA : EBBKC_BATCH_BUILD;
        }
        if (mode == EBBKC_BATCH_BUILD && widest > (uint64_t)(64 * MAX_W)) { delete b; return EBBKC_E_WIDTH; }
    }
    b->build = mode == EBBKC_BATCH_BUILD;
    for (int i = 0; i < n; ++i) {
        ebbkc_graph* g = graphs[i];
        if (ks[i] >= 3 && ks[i] - 2 <= g->tau) {
            if (!b->build) {
                ebbkc_status st = arena_impl(g, s);
                if (st) { delete b; return st; }
            }
        }
        views[(size_t)i] = ArenaView{g->seed_eid, g->seed_c, g->row_off, g->vtx_off, g->arows, g->agid, g->acol};
        bviews[(size_t)i] = BuildGraph{graph_arrays(g), g->subsize,
                                       g->opt.ordering == EBBKC_ORDER_COLOR ? g->vcol : nullptr};
    }
    // graphs whose k exceeds tau + 2 or is below 3 contribute no task
    std::vector<int32_t> kk(b->ks);
    for (int i = 0; i < n; ++i)
        if (kk[(size_t)i] >= 3 && kk[(size_t)i] - 2 > graphs[i]->tau) kk[(size_t)i] = 0;
    b->ks = kk;
    auto fail = [&](ebbkc_status st) { batch_destroy_impl(b); return st; };
    if (dev_alloc(b, (void**)&b->views, sizeof(ArenaView) * n, s) != hipSuccess) return fail(EBBKC_E_OOM);
    if (b->build && dev_alloc(b, (void**)&b->bviews, sizeof(BuildGraph) * n, s) != hipSuccess) return fail(EBBKC_E_OOM);
    if (dev_alloc(b, (void**)&b->gk, sizeof(int32_t) * n, s) != hipSuccess) return fail(EBBKC_E_OOM);
    if (dev_alloc(b, (void**)&b->gtau, sizeof(int32_t) * n, s) != hipSuccess) return fail(EBBKC_E_OOM);
    if (dev_alloc(b, (void**)&b->gtot, sizeof(unsigned long long) * 2 * n, s) != hipSuccess) return fail(EBBKC_E_OOM);
    if (dev_alloc(b, (void**)&b->ctr, sizeof(unsigned long long) * 16, s) != hipSuccess) return fail(EBBKC_E_OOM);
    // the split queue (a few MB) for a batch of its own (served epochs do not
    // split nodes at run time)
    if (!async_mem) {
        if (dev_alloc(b, (void**)&b->squeue, sizeof(SplitItem) * SQ_CAP, s) != hipSuccess ||
            dev_alloc(b, (void**)&b->sq, sizeof(unsigned long long) * SQ_WORDS, s) != hipSuccess)
            return fail(EBBKC_E_OOM);
    }
    if (h_tot && h_ctr) {
        b->own_host = false;
        b->h_tot = h_tot;
        b->h_ctr = h_ctr;
    } else {
        if (hipHostMalloc((void**)&b->h_tot, sizeof(unsigned long long) * 2 * n, hipHostMallocDefault) != hipSuccess)
            return fail(EBBKC_E_OOM);
        if (hipHostMalloc((void**)&b->h_ctr, sizeof(unsigned long long) * 16, hipHostMallocDefault) != hipSuccess)
            return fail(EBBKC_E_OOM);
    }
    std::vector<int32_t> taus((size_t)n);
    for (int i = 0; i < n; ++i) taus[(size_t)i] = graphs[i]->tau;
    if ((b->build && hipMemcpyAsync(b->bviews, bviews.data(), sizeof(BuildGraph) * n, hipMemcpyHostToDevice, s) !=
                         hipSuccess) ||
        hipMemcpyAsync(b->views, views.data(), sizeof(ArenaView) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->gk, b->ks.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->gtau, taus.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(EBBKC_E_HIP);
    if (ensure_tables(b->device, s) != hipSuccess) return fail(EBBKC_E_HIP);
    if (!async_mem) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tune_cache.empty()) load_cache_file();
        auto it = g_tune_cache.find(signature(b));
        if (it != g_tune_cache.end() && !opt) {
            b->opt.split_threshold = it->second.split;
            b->opt.blocks_per_cu = it->second.bpc;
            b->opt.node_split = it->second.node_split;
        }
    }
    ebbkc_status st = build_tasks(b, s);
    if (st) return fail(st);
    *out = b;
    return EBBKC_OK;
}

}  // namespace
}  // namespace ebb

using namespace ebb;

extern "C" {

ebbkc_status ebbkc_batch_create(ebbkc_graph* const* graphs, const int32_t* ks, int32_t n, const ebbkc_options* opt,
                                void* stream, ebbkc_batch** out) {
    if (!graphs || !ks || n <= 0 || !out) return EBBKC_E_INVALID_ARG;
    return batch_create_impl(graphs, ks, n, opt, (hipStream_t)stream, false, nullptr, nullptr, out);
}

ebbkc_status ebbkc_batch_run(ebbkc_batch* b, int32_t use_graph, uint64_t* out_counts, void* stream) {
    if (!b) return EBBKC_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    if (use_graph) {
        if (b->dirty || !b->exec) {
            ebbkc_status st = capture(b, s);
            if (st) return st;
        }
        CHKB(hipGraphLaunch(b->exec, s));
    } else {
        ebbkc_status st = enqueue(b, s);
        if (st) return st;
    }
    CHKB(hipStreamSynchronize(s));
    b->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return finish(b, out_counts);
}

ebbkc_status ebbkc_batch_tune(ebbkc_batch* b, void* stream, int32_t* out_split, int32_t* out_blocks_per_cu,
                              int32_t* out_node_split) {
    if (!b) return EBBKC_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    // tasks that build their g_i are one per seed whatever the threshold
    const std::vector<int32_t> splits = b->build ? std::vector<int32_t>{b->opt.split_threshold}
                                                 : std::vector<int32_t>{1 << 16, 1 << 22, 1 << 28, -1};
    const int32_t bpcs[] = {0, 1, 2, -1};
    const int32_t nsplits[] = {-1, 1 << 16, 0, 1 << 24};  // off, small nodes too .. large ones only (0: 2^20)
    double best = 1e300;
    int32_t bs = b->opt.split_threshold, bb = b->opt.blocks_per_cu, bn = b->opt.node_split;
    std::vector<uint64_t> ref(b->graphs.size()), cur(b->graphs.size());
    bool have_ref = false;
    auto trial = [&](int32_t sp, int32_t bp, int32_t ns) -> ebbkc_status {
        b->opt.blocks_per_cu = bp;
        b->opt.node_split = ns;
        b->dirty = true;
        ebbkc_status st = ebbkc_batch_run(b, 0, cur.data(), stream);
        if (st) return st;
        if (!have_ref) { ref = cur; have_ref = true; }
        else if (cur != ref) return EBBKC_E_HIP;  // every setting must give the same counts
        if (b->last_ms < best) { best = b->last_ms; bs = sp; bb = bp; bn = ns; }
        return EBBKC_OK;
    };
    const int32_t ns0 = b->opt.node_split;
    for (int32_t sp : splits) {
        b->opt.split_threshold = sp;
        ebbkc_status st = build_tasks(b, s);
        if (st) return st;
        for (int32_t bp : bpcs)
            if ((st = trial(sp, bp, ns0))) return st;
    }
    b->opt.split_threshold = bs;
    ebbkc_status st = build_tasks(b, s);
    if (st) return st;
    if (bb != -1)  // the split queue needs persistent grids
        for (int32_t ns : nsplits)
            if (ns != ns0 && (st = trial(bs, bb, ns))) return st;
    b->opt.blocks_per_cu = bb;
    b->opt.node_split = bn;
    b->dirty = true;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[signature(b)] = {bs, bb, bn};
        save_cache_file();
    }
    if (out_split) *out_split = bs;
    if (out_blocks_per_cu) *out_blocks_per_cu = bb;
    if (out_node_split) *out_node_split = bn;
    return EBBKC_OK;
}

ebbkc_status ebbkc_batch_info(const ebbkc_batch* b, int64_t* out_tasks, double* out_last_ms) {
    if (!b) return EBBKC_E_INVALID_ARG;
    if (out_tasks) *out_tasks = b->ntasks;
    if (out_last_ms) *out_last_ms = b->last_ms;
    return EBBKC_OK;
}

void ebbkc_batch_destroy(ebbkc_batch* b) { batch_destroy_impl(b); }

}  // extern "C"

// ============================================================== served form
//
// A catalogue of prepared graphs stays resident; requests (graph, k) are
// submitted as they arrive.  A worker thread keeps up to SLOTS epochs in
// flight, each on its own stream: an epoch takes waiting requests in arrival
// order while the estimated device footprint of all epochs in flight fits the
// budget (a request larger than the budget runs when nothing else does),
// merges their task lists and enqueues one launch per width class.  Each
// launch keeps one workgroup per compute unit fewer than fit, so an epoch
// started on another stream always finds room: requests arriving while a long
// epoch runs start at once in another slot instead of waiting for it.  Device memory of an epoch is stream-ordered, so starting and
// retiring epochs never waits for the device.  Footprint of a request: 16
// bytes per task (task word, graph id, sort key) plus, for each resident wave,
// one c x c bitmap of the graph's largest sub-branch (~tau^2 bits per live
// branch).

#include <condition_variable>
#include <deque>
#include <thread>

namespace {
constexpr int SLOTS = 3;             // the last one takes light requests only
constexpr int SLOT_REQUESTS = 4096;  // most requests in one epoch
constexpr double HEAVY_BOUND = 3e11; // work bound above which a request is heavy
}  // namespace

struct ebbkc_server {
    std::vector<ebbkc_graph*> cat;
    std::vector<int64_t> branch_bytes;  // per graph: tau^2 / 8 bytes
    ebbkc_options opt{};
    int64_t budget = 0;
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        ebbkc_batch* batch = nullptr;
        std::vector<ebbkc_result> reqs;
        int64_t bytes = 0;
        unsigned long long* h_tot = nullptr;  // pinned, 2 * SLOT_REQUESTS
        unsigned long long* h_ctr = nullptr;  // pinned, 16
    } slots[SLOTS];
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    bool stop = false;
    struct Pending {
        ebbkc_result r;
        bool heavy;
        bool solo;  // runs in an epoch of its own (after its shared epoch failed to start)
    };
    std::deque<Pending> pending;
    std::vector<ebbkc_result> done;
    std::vector<int64_t> cancelled;  // ids of running requests whose result is withdrawn
    std::set<int64_t> running;       // ids admitted to an epoch and not yet retired (under mu)
    std::vector<std::vector<int64_t>> chist;  // per graph: seeds by |V(g_i)| (0..256)
    int64_t next_id = 0, in_flight = 0, epochs = 0, max_epoch_requests = 0, in_flight_bytes = 0;
    std::chrono::steady_clock::time_point t0;
    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace ebb {
namespace {

int64_t request_bytes(const ebbkc_server* S, const ebbkc_result& r) {
    const ebbkc_graph* g = S->cat[(size_t)r.graph];
    const int64_t waves = 4096;  // resident waves of a launch (upper bound)
    return 16 * (g->nseeds + 1) + waves * S->branch_bytes[(size_t)r.graph];
}

// Bound on the search of request (graph, k): sum over the seeds of
// C(|V(g_i)|, k-2), the (k-2)-subsets a root could extend.  Loose (closed
// forms end dense branches early) but it separates the requests that run for
// seconds from those that take a millisecond.
bool is_heavy(const ebbkc_server* S, int32_t graph, int32_t k) {
    if (k < 5) return false;
    const std::vector<int64_t>& h = S->chist[(size_t)graph];
    double b = 0.0;
    for (int c = k - 2; c < (int)h.size(); ++c)
        if (h[(size_t)c]) b += (double)h[(size_t)c] * std::exp(std::lgamma(c + 1.0) - std::lgamma(k - 1.0) - std::lgamma(c - k + 3.0));
    return b > HEAVY_BOUND;
}

// Finish the epoch of slot sl (its event has completed): results to done.
void retire(ebbkc_server* S, ebbkc_server::Slot& sl) {
    std::vector<uint64_t> cnt(sl.reqs.size(), 0);
    std::vector<ebbkc_status> sts(sl.reqs.size(), EBBKC_OK);
    (void)finish(sl.batch, cnt.data(), sts.data());
    batch_destroy_impl(sl.batch);
    sl.batch = nullptr;
    const double t_done = S->now_ms();
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        ebbkc_result r = sl.reqs[i];
        r.status = sts[i];
        S->running.erase(r.id);
        auto ci = std::find(S->cancelled.begin(), S->cancelled.end(), r.id);
        if (ci != S->cancelled.end()) {
            S->cancelled.erase(ci);
            r.status = EBBKC_E_CANCELLED;
        }
        r.count = r.status ? 0 : cnt[i];
        r.done_ms = t_done;
        S->done.push_back(r);
    }
    S->in_flight -= (int64_t)sl.reqs.size();
    S->in_flight_bytes -= sl.bytes;
    S->epochs++;
    sl.reqs.clear();
    sl.bytes = 0;
}

void serve_loop(ebbkc_server* S) {
    (void)hipSetDevice(S->cat.empty() ? 0 : S->cat[0]->device);
    for (;;) {
        bool progressed = false;
        for (auto& sl : S->slots) {
            if (sl.batch && hipEventQuery(sl.done) == hipSuccess) {
                retire(S, sl);
                progressed = true;
            }
        }
        if (progressed) S->done_cv.notify_all();
        // admit waiting requests: every free slot takes the requests of one
        // class (heavy or light, the class of the oldest waiting request; the
        // last slot light only) in arrival order while the footprint of the
        // epochs in flight fits the budget
        int busy = 0;
        for (auto& sl : S->slots) busy += sl.batch != nullptr;
        struct Start {
            ebbkc_server::Slot* slot;
            std::vector<ebbkc_result> reqs;
            int64_t bytes;
            bool solo;
        };
        std::vector<Start> starts;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop && S->pending.empty() && busy == 0) return;
            for (int si = 0; si < SLOTS && !S->pending.empty(); ++si) {
                ebbkc_server::Slot& sl = S->slots[si];
                if (sl.batch) continue;
                const bool light_only = si == SLOTS - 1;
                bool heavy = light_only ? false : S->pending.front().heavy;
                Start st{&sl, {}, 0, false};
                for (auto it = S->pending.begin(); it != S->pending.end() && (int)st.reqs.size() < SLOT_REQUESTS;) {
                    if (it->heavy != heavy) { ++it; continue; }
                    if (it->solo && !st.reqs.empty()) break;
                    const int64_t need = request_bytes(S, it->r);
                    const bool alone = st.reqs.empty() && busy == 0 && starts.empty();
                    if (!alone && S->in_flight_bytes + st.bytes + need > S->budget) break;
                    st.bytes += need;
                    st.reqs.push_back(it->r);
                    S->running.insert(it->r.id);
                    st.solo = it->solo;
                    it = S->pending.erase(it);
                    if (st.solo) break;
                }
                if (st.reqs.empty()) continue;
                S->in_flight += (int64_t)st.reqs.size();
                S->in_flight_bytes += st.bytes;
                S->max_epoch_requests = std::max<int64_t>(S->max_epoch_requests, (int64_t)st.reqs.size());
                starts.push_back(std::move(st));
            }
            if (starts.empty() && !progressed) {
                // nothing to start: wait for a submission, or poll the epochs in flight
                if (busy == 0) S->cv.wait(lk, [&] { return S->stop || !S->pending.empty(); });
                else S->cv.wait_for(lk, std::chrono::microseconds(50));
                continue;
            }
        }
        for (auto& start : starts) {
            std::vector<ebbkc_result>& epoch = start.reqs;
            ebbkc_server::Slot* free_slot = start.slot;
            const int64_t bytes = start.bytes;
            const double t_admit = S->now_ms();
            std::vector<ebbkc_graph*> gs;
            std::vector<int32_t> ks;
            for (auto& r : epoch) {
                r.admit_ms = t_admit;
                gs.push_back(S->cat[(size_t)r.graph]);
                ks.push_back(r.k);
            }
            ebbkc_server::Slot& sl = *free_slot;
            sl.reqs = epoch;
            sl.bytes = bytes;
            ebbkc_options o = S->opt;
            o.blocks_per_cu = -2;  // leave room on every CU for the epochs of the other slots
            ebbkc_batch* b = nullptr;
            ebbkc_status st = batch_create_impl(gs.data(), ks.data(), (int32_t)gs.size(), &o, sl.stream, true, sl.h_tot,
                                                sl.h_ctr, &b);
            if (!st) st = enqueue(b, sl.stream);
            if (!st && hipEventRecord(sl.done, sl.stream) != hipSuccess) st = EBBKC_E_HIP;
            if (st) {
                if (b) {
                    (void)hipStreamSynchronize(sl.stream);
                    batch_destroy_impl(b);
                }
                const double t_done = S->now_ms();
                std::lock_guard<std::mutex> lk(S->mu);
                for (auto& r : sl.reqs) S->running.erase(r.id);
                if (sl.reqs.size() > 1) {
                    // an epoch of several requests that could not start (device
                    // memory, a runtime error) goes back to the front of the
                    // queue one request per epoch, so a request that cannot
                    // run fails alone and its neighbours still get results
                    for (auto it = sl.reqs.rbegin(); it != sl.reqs.rend(); ++it)
                        S->pending.push_front({*it, is_heavy(S, it->graph, it->k), true});
                } else {
                    for (auto& r : sl.reqs) {
                        auto ci = std::find(S->cancelled.begin(), S->cancelled.end(), r.id);
                        if (ci != S->cancelled.end()) S->cancelled.erase(ci);
                        r.status = st;
                        r.count = 0;
                        r.done_ms = t_done;
                        S->done.push_back(r);
                    }
                    S->epochs++;
                }
                S->in_flight -= (int64_t)sl.reqs.size();
                S->in_flight_bytes -= sl.bytes;
                sl.reqs.clear();
                sl.bytes = 0;
                S->done_cv.notify_all();
                continue;
            }
            sl.batch = b;
        }
    }
}

void server_free(ebbkc_server* S) {
    for (auto& sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.h_tot) (void)hipHostFree(sl.h_tot);
        if (sl.h_ctr) (void)hipHostFree(sl.h_ctr);
    }
    delete S;
}

}  // namespace
}  // namespace ebb

extern "C" {

ebbkc_status ebbkc_server_create(ebbkc_graph* const* graphs, int32_t n, const ebbkc_options* opt, int64_t budget_bytes,
                                 ebbkc_server** out) {
    if (!graphs || n <= 0 || !out || budget_bytes <= 0) return EBBKC_E_INVALID_ARG;
    ebbkc_server* S = new ebbkc_server();
    S->cat.assign(graphs, graphs + n);
    if (opt) S->opt = *opt; else ebbkc_default_options(&S->opt);
    S->opt.count_work = 0;
    S->budget = budget_bytes;
    for (int i = 0; i < n; ++i) {
        if (!graphs[i]) { delete S; return EBBKC_E_INVALID_ARG; }
        const int64_t t = graphs[i]->tau + 2;
        S->branch_bytes.push_back((t * t + 7) / 8);
        std::vector<int64_t> h(257, 0);
        if (graphs[i]->tau >= 1) {
            ebbkc_status st = ebb::arena_impl(graphs[i], nullptr);  // resident before the first request
            if (st) { delete S; return st; }
            std::vector<int32_t> sc((size_t)graphs[i]->nseeds);
            if (!sc.empty() &&
                hipMemcpy(sc.data(), graphs[i]->seed_c, sizeof(int32_t) * sc.size(), hipMemcpyDeviceToHost) != hipSuccess) {
                delete S;
                return EBBKC_E_HIP;
            }
            for (int32_t c : sc) h[(size_t)std::min(c, 256)]++;
        }
        S->chist.push_back(std::move(h));
    }
    if (ebb::ensure_tables(graphs[0]->device, nullptr) != hipSuccess) { delete S; return EBBKC_E_HIP; }
    for (auto& sl : S->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&sl.h_tot, sizeof(unsigned long long) * 2 * SLOT_REQUESTS, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void**)&sl.h_ctr, sizeof(unsigned long long) * 16, hipHostMallocDefault) != hipSuccess) {
            ebb::server_free(S);
            return EBBKC_E_HIP;
        }
    }
    S->t0 = std::chrono::steady_clock::now();
    S->worker = std::thread(ebb::serve_loop, S);
    *out = S;
    return EBBKC_OK;
}

ebbkc_status ebbkc_server_submit(ebbkc_server* S, int32_t graph, int32_t k, int64_t* out_id) {
    if (!S || graph < 0 || graph >= (int32_t)S->cat.size() || k < 1) return EBBKC_E_INVALID_ARG;
    if (k > ebb::MAX_K) return EBBKC_E_K_RANGE;
    ebbkc_result r{};
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r.id = S->next_id++;
        r.graph = graph;
        r.k = k;
        r.arrival_ms = S->now_ms();
        S->pending.push_back({r, ebb::is_heavy(S, graph, k), false});
    }
    S->cv.notify_one();
    if (out_id) *out_id = r.id;
    return EBBKC_OK;
}

ebbkc_status ebbkc_server_cancel(ebbkc_server* S, int64_t id) {
    if (!S || id < 0) return EBBKC_E_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (id >= S->next_id) return EBBKC_E_INVALID_ARG;
        for (auto it = S->pending.begin(); it != S->pending.end(); ++it) {
            if (it->r.id != id) continue;
            ebbkc_result r = it->r;
            S->pending.erase(it);
            r.status = EBBKC_E_CANCELLED;
            r.count = 0;
            r.admit_ms = r.done_ms = S->now_ms();
            S->done.push_back(r);
            S->done_cv.notify_all();
            return EBBKC_OK;
        }
        if (S->running.count(id)) {
            if (std::find(S->cancelled.begin(), S->cancelled.end(), id) == S->cancelled.end())
                S->cancelled.push_back(id);
            return EBBKC_OK;
        }
    }
    return EBBKC_E_INVALID_ARG;  // finished already
}

ebbkc_status ebbkc_server_poll(ebbkc_server* S, ebbkc_result* out, int32_t max, int32_t wait, int32_t* n_out) {
    if (!S || !n_out || (max > 0 && !out)) return EBBKC_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    if (wait) S->done_cv.wait(lk, [&] { return !S->done.empty() || (S->pending.empty() && S->in_flight == 0); });
    const int32_t n = (int32_t)std::min<size_t>((size_t)max, S->done.size());
    for (int32_t i = 0; i < n; ++i) out[i] = S->done[(size_t)i];
    S->done.erase(S->done.begin(), S->done.begin() + n);
    *n_out = n;
    return EBBKC_OK;
}

ebbkc_status ebbkc_server_stats(const ebbkc_server* S, int64_t out[4]) {
    if (!S || !out) return EBBKC_E_INVALID_ARG;
    ebbkc_server* M = const_cast<ebbkc_server*>(S);
    std::lock_guard<std::mutex> lk(M->mu);
    out[0] = S->next_id;
    out[1] = S->epochs;
    out[2] = S->max_epoch_requests;
    out[3] = (int64_t)S->pending.size() + S->in_flight;
    return EBBKC_OK;
}

void ebbkc_server_destroy(ebbkc_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    ebb::server_free(S);
}

}  // extern "C"
