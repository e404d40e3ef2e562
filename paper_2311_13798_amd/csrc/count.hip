// count.hip -- host orchestration of counting: the sub-branch arena, task
// generation and the per-width-class search launches.
//
// Seeds.  Every k-clique is counted under the edge of the clique that comes
// first in pi_tau (Section 4.1), inside that edge's sub-branch g_i, which
// needs at least k-2 vertices.  The arena keeps g_i for every edge with
// |V(g_i)| >= 1, in rank order, so a rank range is a slot range.
//
// Tasks.  For a count at k, every slot with |V(g_i)| >= k-2 becomes one task;
// a slot whose root has more than split_threshold (k-2)-subsets becomes one
// task per possible first vertex x of the root's children.  Tasks are sorted
// by bitmap width class, and inside a class by the number of vertices the
// task's subtree can still use, largest first, so heavy work starts first.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "arena.h"
#include "common.h"
#include "handle.h"
#include "prims.h"

namespace ebb {

namespace {

std::once_flag g_binom_once[64];
hipError_t g_binom_err[64];

hipError_t ensure_binom(int dev, hipStream_t s) {
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::call_once(g_binom_once[dev], [&] {
        g_binom_err[dev] = launch_binom_init(s);
        if (g_binom_err[dev] == hipSuccess) g_binom_err[dev] = hipStreamSynchronize(s);
    });
    return g_binom_err[dev];
}

int opts_of(const ebbkc_options& o) {
    int f = 0;
    if (o.early_termination) f |= OPT_ET;
    if (o.rule1) f |= OPT_RULE1;
    if (o.rule2) f |= OPT_RULE2;
    if (o.count_work) f |= OPT_WORK;
    return f;
}

// counters: [0..4) per-class work queues, [4,5] total lo/hi, [6] error flags,
// [12..16) per-class task counts (task generation), [16 + 4 (W-1) ..) search
// work of width class W (tasks, nodes, word operations), [32 + 4 (W-1) ..)
// its waves' end times (sum, latest, count, ~earliest start), [48 + W-1]
// nodes it handed over through the split queue
constexpr int CNT_WORDS = 64;

GraphView graph_view(const ebbkc_graph* g) {
    return GraphView{g->rp, g->ci, g->erank, g->rrow, g->orp, g->orow, g->eu, g->ev, g->rank,
                     g->adj, g->acum, g->adjw};
}

__host__ __device__ inline int width_of(int c) { return c <= 64 ? 1 : (c <= 128 ? 2 : (c <= 192 ? 3 : 4)); }

inline unsigned grid_for(int64_t n, int per = 256) {
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (unsigned)b;
}

// ---------------------------------------------------------------- kernels

__global__ void k_seed_flags(const int32_t* __restrict__ byrank, const int32_t* __restrict__ subsize, int64_t m,
                             int32_t* __restrict__ flag) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x)
        flag[r] = subsize[byrank[r]] >= 1;
}

__global__ void k_seed_fill(const int32_t* __restrict__ byrank, const int32_t* __restrict__ subsize,
                            const int32_t* __restrict__ flag, const int64_t* __restrict__ pos, int64_t m,
                            int32_t* __restrict__ seed_eid, int32_t* __restrict__ seed_c,
                            int32_t* __restrict__ seed_rank, int64_t* __restrict__ rwords,
                            int64_t* __restrict__ vcount, int* __restrict__ err) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[r]) continue;
        const int64_t s = pos[r];
        const int32_t e = byrank[r], c = subsize[e];
        if (c > 64 * MAX_W) atomicOr(err, ERR_WIDTH);
        seed_eid[s] = e;
        seed_c[s] = c;
        seed_rank[s] = (int32_t)r;
        rwords[s] = (int64_t)c * width_of(c);
        vcount[s] = c;
    }
}

// node-parallel roots: |N+(v)| (neighbours later in the vertex order) per vertex
__global__ void k_vertex_out(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const int32_t* __restrict__ vpos, int32_t n, int32_t* __restrict__ cout,
                             int32_t* __restrict__ byvpos) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t pv = vpos[v];
        int32_t c = 0;
        for (int32_t j = rp[v]; j < rp[v + 1]; ++j) c += vpos[ci[j]] > pv;
        cout[pv] = c;  // indexed by position
        byvpos[pv] = (int32_t)v;
    }
}

__global__ void k_vertex_flags(const int32_t* __restrict__ cout, int32_t n, int32_t* __restrict__ flag) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        flag[p] = cout[p] >= 1;
}

// slot of the vertex at position p: its out-edges are the ranks [R, R + c) (edges are ranked
// lexicographically by their endpoints' positions), so its sub-branch is the neighbourhood through
// edges ranked after R - 1
__global__ void k_vertex_fill(const int32_t* __restrict__ cout, const int32_t* __restrict__ byvpos,
                              const int64_t* __restrict__ rstart, const int32_t* __restrict__ flag,
                              const int64_t* __restrict__ pos, int32_t n, int32_t* __restrict__ seed_v,
                              int32_t* __restrict__ seed_c, int32_t* __restrict__ seed_rthr,
                              int32_t* __restrict__ seed_rank, int64_t* __restrict__ rwords,
                              int64_t* __restrict__ vcount, int* __restrict__ err) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[p]) continue;
        const int64_t s = pos[p];
        const int32_t c = cout[p];
        if (c > 64 * MAX_W) atomicOr(err, ERR_WIDTH);
        seed_v[s] = byvpos[p];
        seed_c[s] = c;
        seed_rthr[s] = (int32_t)(rstart[p] - 1);
        seed_rank[s] = (int32_t)rstart[p];
        rwords[s] = (int64_t)c * width_of(c);
        vcount[s] = c;
    }
}

// slots of one width class, in slot order
__global__ void k_class_flags(const int32_t* __restrict__ seed_c, int64_t n, int W, int32_t* __restrict__ flag) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        flag[s] = width_of(seed_c[s]) == W;
}

__global__ void k_class_fill(const int32_t* __restrict__ flag, const int64_t* __restrict__ pos, int64_t n,
                             int32_t* __restrict__ list) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        if (flag[s]) list[pos[s]] = (int32_t)s;
}

__global__ void k_task_counts(const int32_t* __restrict__ seed_c, int64_t i0, int64_t n, int l0, double log_thr,
                              int32_t* __restrict__ tcount) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = seed_c[i0 + i];
        tcount[i] = c >= l0 ? root_tasks(c, l0, log_thr, [](int, int) {}) : 0;
    }
}

__global__ void k_task_fill(const int32_t* __restrict__ seed_c, int64_t i0, int64_t n, int l0, double log_thr,
                            const int64_t* __restrict__ toff, int64_t* __restrict__ tasks, uint64_t* __restrict__ keys,
                            uint32_t* __restrict__ vals, unsigned long long* __restrict__ cls_count) {
    uint64_t per_class[4] = {0, 0, 0, 0};  // tasks per width class, added once per wave below
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = seed_c[i0 + i];
        if (c < l0) continue;
        const int W = width_of(c);
        int64_t o = toff[i];
        const int nt = root_tasks(c, l0, log_thr, [&](int x0, int x1) {
            tasks[o] = task_pack(i0 + i, x0, x1);
            // heaviest first: more vertices after the first one of the range
            const int usable = x0 == 0 && x1 >= c ? c : c - 1 - x0;
            keys[o] = ((uint64_t)(W - 1) << 8) | (uint64_t)(255 - (usable > 255 ? 255 : usable));
            vals[o] = (uint32_t)o;
            ++o;
        });
#pragma unroll
        for (int w = 0; w < 4; ++w) per_class[w] += w == W - 1 ? (uint64_t)nt : 0;
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint64_t t = wave_sum(per_class[w]);
        if (lane_id() == 0 && t) atomicAdd(&cls_count[w], (unsigned long long)t);
    }
}

__global__ void k_gather_tasks(const int64_t* __restrict__ tasks, const uint32_t* __restrict__ idx, int64_t n,
                               int64_t* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = tasks[idx[i]];
}

// sum of a per-item value over [lo, hi): k = 3 sums |V(g_i)| by rank, k = 4 |E(g_i)| by slot
__global__ void k_sum_range(const int32_t* __restrict__ byrank, const int32_t* __restrict__ vals32,
                            const uint64_t* __restrict__ vals64, int64_t lo, int64_t hi,
                            unsigned long long* __restrict__ out) {
    uint64_t acc = 0;
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (int64_t)gridDim.x * blockDim.x)
        acc += vals32 ? (uint64_t)vals32[byrank ? byrank[i] : i] : vals64[i];
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(out, (unsigned long long)acc);
}

// bump allocator over one scratch buffer
struct Carve {
    char* base;
    size_t used, cap;
    template <typename T>
    T* take(int64_t n) {
        const size_t bytes = ((sizeof(T) * (size_t)(n > 0 ? n : 1)) + 255) & ~(size_t)255;
        if (!base || used + bytes > cap) return nullptr;
        T* p = reinterpret_cast<T*>(base + used);
        used += bytes;
        return p;
    }
};

inline size_t rnd256(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename T>
struct DBuf {
    T* p = nullptr;
    hipError_t alloc(int64_t n) { return hipMalloc((void**)&p, sizeof(T) * (size_t)(n > 0 ? n : 1)); }
    ~DBuf() { if (p) (void)hipFree(p); }
    T* release() { T* q = p; p = nullptr; return q; }
};

struct SlotArrays {
    uint64_t* rows = nullptr;
    int32_t* gid = nullptr;
    int16_t* col = nullptr;
    uint64_t* ned = nullptr;
};

}  // namespace

hipError_t ensure_tables(int dev, hipStream_t s) { return ensure_binom(dev, s); }

#define CHKH(expr)                                                              \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) {                                                 \
            (void)hipGetLastError();                                            \
            return e_ == hipErrorOutOfMemory ? EBBKC_E_OOM : EBBKC_E_HIP;       \
        }                                                                       \
    } while (0)

void* scratch_get(ebbkc_graph* g, size_t bytes) {
    if (bytes <= g->scratch_bytes) return g->scratch;
    if (g->scratch) (void)hipFree(g->scratch);
    g->scratch = nullptr;
    g->scratch_bytes = 0;
    const size_t nb = bytes + bytes / 4;
    if (hipMalloc(&g->scratch, nb) != hipSuccess) return nullptr;
    g->scratch_bytes = nb;
    return g->scratch;
}

static ebbkc_status ensure_counters(ebbkc_graph* g) {
    if (!g->d_counters) {
        if (hipMalloc((void**)&g->d_counters, CNT_WORDS * sizeof(uint64_t)) != hipSuccess) return EBBKC_E_OOM;
        if (hipHostMalloc((void**)&g->h_counters, CNT_WORDS * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess)
            return EBBKC_E_OOM;
    }
    return EBBKC_OK;
}

ebbkc_status subsize_impl(ebbkc_graph* g, hipStream_t s) {
    if (g->subsize_ready) return EBBKC_OK;
    if (!g->subsize && hipMalloc((void**)&g->subsize, sizeof(int32_t) * (size_t)(g->m > 0 ? g->m : 1)) != hipSuccess)
        return EBBKC_E_OOM;
    CHKH(launch_subsize(graph_view(g), g->m, g->subsize, s));
    g->subsize_ready = true;
    return EBBKC_OK;
}

static ebbkc_status build_slots(ebbkc_graph* g, int64_t ns, const int32_t* seid, const int32_t* sc,
                                const int32_t* srthr, const int64_t* roff, const int64_t* voff, const int64_t tot[2],
                                int64_t* tmp, SlotArrays& out, hipStream_t s);

ebbkc_status arena_impl(ebbkc_graph* g, hipStream_t s) {
    if (g->arena_built) return EBBKC_OK;
    ebbkc_status st = ensure_counters(g);
    if (st) return st;
    hipEvent_t e0, e1;
    CHKH(hipEventCreate(&e0));
    CHKH(hipEventCreate(&e1));
    CHKH(hipEventRecord(e0, s));
    st = subsize_impl(g, s);
    if (st) return st;
    const int64_t m = g->m;
    DBuf<int32_t> flag, srank;
    DBuf<int64_t> pos, tmp, rwords, vcount;
    CHKH(flag.alloc(m));
    CHKH(pos.alloc(m + 1));
    CHKH(tmp.alloc(scan_tmp_elems(m + 1) + 64));
    CHKH(hipMemsetAsync(g->d_counters, 0, CNT_WORDS * sizeof(uint64_t), s));
    int* err = (int*)(g->d_counters + 6);
    if (m) hipLaunchKernelGGL(k_seed_flags, dim3(grid_for(m)), dim3(256), 0, s, g->byrank, g->subsize, m, flag.p);
    CHKH(exclusive_scan_i32(flag.p, pos.p, m, pos.p + m, tmp.p, s));
    int64_t ns = 0;
    CHKH(hipMemcpyAsync(&ns, pos.p + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    DBuf<int32_t> seid, sc;
    DBuf<int64_t> roff, voff;
    CHKH(seid.alloc(ns));
    CHKH(sc.alloc(ns));
    CHKH(srank.alloc(ns));
    CHKH(rwords.alloc(ns + 1));
    CHKH(vcount.alloc(ns + 1));
    CHKH(roff.alloc(ns + 1));
    CHKH(voff.alloc(ns + 1));
    if (m)
        hipLaunchKernelGGL(k_seed_fill, dim3(grid_for(m)), dim3(256), 0, s, g->byrank, g->subsize, flag.p, pos.p, m,
                           seid.p, sc.p, srank.p, rwords.p, vcount.p, err);
    CHKH(exclusive_scan_i64(rwords.p, roff.p, ns, roff.p + ns, tmp.p, s));
    CHKH(exclusive_scan_i64(vcount.p, voff.p, ns, voff.p + ns, tmp.p, s));
    int64_t tot[2] = {0, 0};
    int herr = 0;
    CHKH(hipMemcpyAsync(&tot[0], roff.p + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipMemcpyAsync(&tot[1], voff.p + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    g->seed_rank_host.resize((size_t)ns);
    if (ns) CHKH(hipMemcpyAsync(g->seed_rank_host.data(), srank.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    if (herr & ERR_WIDTH) return EBBKC_E_WIDTH;
    SlotArrays out;
    st = build_slots(g, ns, seid.p, sc.p, nullptr, roff.p, voff.p, tot, tmp.p, out, s);
    if (st) return st;
    CHKH(hipEventRecord(e1, s));
    CHKH(hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g->arena_ms = ms;
    g->nseeds = ns;
    g->seed_eid = seid.release();
    g->seed_c = sc.release();
    g->row_off = roff.release();
    g->vtx_off = voff.release();
    g->arows = out.rows;
    g->agid = out.gid;
    g->acol = out.col;
    g->nedges = out.ned;
    g->arena_bytes = (int64_t)(tot[0] * 8 + tot[1] * 6 + ns * 32);
    g->device_bytes += g->arena_bytes;
    g->arena_built = true;
    return EBBKC_OK;
}

// The sub-branches of ns slots -- seed edges (srthr null) or vertices with
// the rank threshold of their out-edges -- built per width class into newly
// allocated rows / gid / col / nedges (owned by the caller on success).
static ebbkc_status build_slots(ebbkc_graph* g, int64_t ns, const int32_t* seid, const int32_t* sc,
                                const int32_t* srthr, const int64_t* roff, const int64_t* voff, const int64_t tot[2],
                                int64_t* tmp, SlotArrays& out, hipStream_t s) {
    int* err = (int*)(g->d_counters + 6);
    int herr = 0;
    DBuf<uint64_t> rows, ned;
    DBuf<int32_t> gid;
    DBuf<int16_t> col;
    CHKH(rows.alloc(tot[0]));
    CHKH(gid.alloc(tot[1]));
    CHKH(col.alloc(tot[1]));
    CHKH(ned.alloc(ns));
    // per width class: the slot list, then the build kernel
    DBuf<int32_t> cflag, clist;
    DBuf<int64_t> cpos;
    CHKH(cflag.alloc(ns));
    CHKH(clist.alloc(ns));
    CHKH(cpos.alloc(ns + 1));
    for (int W = MAX_W; W >= 1 && ns > 0; --W) {
        hipLaunchKernelGGL(k_class_flags, dim3(grid_for(ns)), dim3(256), 0, s, sc, ns, W, cflag.p);
        CHKH(exclusive_scan_i32(cflag.p, cpos.p, ns, cpos.p + ns, tmp, s));
        hipLaunchKernelGGL(k_class_fill, dim3(grid_for(ns)), dim3(256), 0, s, cflag.p, cpos.p, ns, clist.p);
        int64_t nw = 0;
        CHKH(hipMemcpyAsync(&nw, cpos.p + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CHKH(hipStreamSynchronize(s));
        if (!nw) continue;
        CHKH(hipMemsetAsync(g->d_counters + W - 1, 0, sizeof(uint64_t), s));
        BuildArgs b{};
        b.G = graph_view(g);
        b.list = clist.p;
        b.n = nw;
        b.seed_eid = seid;
        b.seed_c = sc;
        b.seed_rthr = srthr;
        b.row_off = roff;
        b.vtx_off = voff;
        b.rows = rows.p;
        b.gid = gid.p;
        b.col = col.p;
        b.nedges = ned.p;
        b.vcol = g->opt.ordering == EBBKC_ORDER_COLOR ? g->vcol : nullptr;
        b.next = (unsigned long long*)(g->d_counters + W - 1);
        b.err = err;
        CHKH(launch_build(W, b, g->cu_count, s));
        CHKH(hipStreamSynchronize(s));  // clist is reused by the next class
    }
    CHKH(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    if (herr & ERR_WIDTH) return EBBKC_E_WIDTH;
    out.rows = rows.release();
    out.gid = gid.release();
    out.col = col.release();
    out.ned = ned.release();
    return EBBKC_OK;
}

// Node-parallel VBBkC (ordering DEGEN_VERTEX_NP): one slot per vertex v with a
// non-empty N+(v) (neighbours later in the degeneracy order), its sub-branch
// G[N+(v)] built by the same kernel (the neighbourhood through edges ranked
// after v's first out-edge, all edges among it), in position order.
static ebbkc_status vertex_arena_impl(ebbkc_graph* g, hipStream_t s) {
    VertexArena& A = g->varena;
    if (A.built) return EBBKC_OK;
    ebbkc_status st = ensure_counters(g);
    if (st) return st;
    const int32_t n = g->n;
    DBuf<int32_t> cout, byvpos, flag, seid, sc, srthr, srank;
    DBuf<int64_t> rstart, pos, tmp, rwords, vcount, roff, voff;
    CHKH(cout.alloc(n));
    CHKH(byvpos.alloc(n));
    CHKH(flag.alloc(n));
    CHKH(rstart.alloc(n + 1));
    CHKH(pos.alloc(n + 1));
    CHKH(tmp.alloc(scan_tmp_elems(n + 1) + 64));
    CHKH(hipMemsetAsync(g->d_counters, 0, CNT_WORDS * sizeof(uint64_t), s));
    int* err = (int*)(g->d_counters + 6);
    if (n) {
        hipLaunchKernelGGL(k_vertex_out, dim3(grid_for(n)), dim3(256), 0, s, g->rp, g->ci, g->vpos, n, cout.p,
                           byvpos.p);
        hipLaunchKernelGGL(k_vertex_flags, dim3(grid_for(n)), dim3(256), 0, s, cout.p, n, flag.p);
    }
    CHKH(exclusive_scan_i32(cout.p, rstart.p, n, rstart.p + n, tmp.p, s));
    CHKH(exclusive_scan_i32(flag.p, pos.p, n, pos.p + n, tmp.p, s));
    int64_t ns = 0;
    CHKH(hipMemcpyAsync(&ns, pos.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    CHKH(seid.alloc(ns));
    CHKH(sc.alloc(ns));
    CHKH(srthr.alloc(ns));
    CHKH(srank.alloc(ns));
    CHKH(rwords.alloc(ns + 1));
    CHKH(vcount.alloc(ns + 1));
    CHKH(roff.alloc(ns + 1));
    CHKH(voff.alloc(ns + 1));
    if (n)
        hipLaunchKernelGGL(k_vertex_fill, dim3(grid_for(n)), dim3(256), 0, s, cout.p, byvpos.p, rstart.p, flag.p,
                           pos.p, n, seid.p, sc.p, srthr.p, srank.p, rwords.p, vcount.p, err);
    CHKH(exclusive_scan_i64(rwords.p, roff.p, ns, roff.p + ns, tmp.p, s));
    CHKH(exclusive_scan_i64(vcount.p, voff.p, ns, voff.p + ns, tmp.p, s));
    int64_t tot[2] = {0, 0};
    int herr = 0;
    CHKH(hipMemcpyAsync(&tot[0], roff.p + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipMemcpyAsync(&tot[1], voff.p + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<int32_t> rank_host((size_t)ns);
    if (ns) CHKH(hipMemcpyAsync(rank_host.data(), srank.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    if (herr & ERR_WIDTH) return EBBKC_E_WIDTH;
    SlotArrays out;
    st = build_slots(g, ns, seid.p, sc.p, srthr.p, roff.p, voff.p, tot, tmp.p, out, s);
    if (st) return st;
    A.nseeds = ns;
    A.seed_v = seid.release();
    A.seed_c = sc.release();
    A.seed_rthr = srthr.release();
    A.row_off = roff.release();
    A.vtx_off = voff.release();
    A.rows = out.rows;
    A.gid = out.gid;
    A.col = out.col;
    A.nedges = out.ned;
    A.rank_host.swap(rank_host);
    A.bytes = (int64_t)(tot[0] * 8 + tot[1] * 6 + ns * 36);
    g->device_bytes += A.bytes;
    A.built = true;
    return EBBKC_OK;
}

// exchange the edge arena of the handle with its vertex arena
static void swap_arenas(ebbkc_graph* g) {
    VertexArena& A = g->varena;
    std::swap(g->nseeds, A.nseeds);
    std::swap(g->seed_eid, A.seed_v);
    std::swap(g->seed_c, A.seed_c);
    std::swap(g->row_off, A.row_off);
    std::swap(g->vtx_off, A.vtx_off);
    std::swap(g->arows, A.rows);
    std::swap(g->agid, A.gid);
    std::swap(g->acol, A.col);
    std::swap(g->nedges, A.nedges);
    std::swap(g->seed_rank_host, A.rank_host);
    std::swap(g->arena_built, A.built);
    g->np_active = !g->np_active;
}

static ebbkc_status read_total(ebbkc_graph* g, uint64_t* out, hipStream_t s) {
    CHKH(hipMemcpyAsync(g->h_counters, g->d_counters, CNT_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    const int err = (int)g->h_counters[6];
    if (err & ERR_WIDTH) return EBBKC_E_WIDTH;
    if (err & ERR_DEPTH) return EBBKC_E_K_RANGE;
    if (err & ERR_QUEUE) return EBBKC_E_HIP;
    // the exact total is 128 bits wide; the 64-bit result is an error past 2^64
    g->last_total[0] = g->h_counters[4];
    g->last_total[1] = g->h_counters[5];
    g->last_total_ovf = (err & ERR_OVERFLOW) != 0;
    if ((err & ERR_OVERFLOW) || g->h_counters[5] != 0) return EBBKC_E_OVERFLOW;
    *out = g->h_counters[4];
    for (int i = 0; i < 4; ++i) g->last_work[i] = 0;
    for (int W = 1; W <= 4; ++W) {
        for (int i = 0; i < 3; ++i) {
            g->last_work_class[W - 1][i] = g->h_counters[16 + 4 * (W - 1) + i];
            g->last_work[i] += g->last_work_class[W - 1][i];
        }
        // wave-finish tail: latest end minus the mean end (10 ns ticks)
        const uint64_t* t = g->h_counters + 32 + 4 * (W - 1);
        g->last_work_class[W - 1][3] = t[2] ? 10 * (t[1] - t[0] / t[2]) : 0;
        g->last_work[3] += g->h_counters[48 + W - 1];
    }
    return EBBKC_OK;
}

// Task list of slots [i0, i1) at l0 = k-2, sorted (width class, heaviest
// first) into `sorted`; class sizes into ccount.  Scratch comes from cv.
static ebbkc_status make_tasks(ebbkc_graph* g, int64_t i0, int64_t n, int l0, double log_thr, hipStream_t s,
                               Carve& cv, int64_t** sorted, int64_t* T_out, uint64_t ccount[4]) {
    int32_t* tcount = cv.take<int32_t>(n);
    int64_t* toff = cv.take<int64_t>(n + 1);
    int64_t* tmp = cv.take<int64_t>(scan_tmp_elems(n + 1) + 64);
    if (!tcount || !toff || !tmp) return EBBKC_E_OOM;
    hipLaunchKernelGGL(k_task_counts, dim3(grid_for(n)), dim3(256), 0, s, g->seed_c, i0, n, l0, log_thr, tcount);
    CHKH(exclusive_scan_i32(tcount, toff, n, toff + n, tmp, s));
    int64_t T = 0;
    CHKH(hipMemcpyAsync(&T, toff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    *T_out = T;
    if (T == 0) return EBBKC_OK;
    if (T >= ((int64_t)1 << 32)) return EBBKC_E_OOM;
    const int64_t hn = radix_hist_elems(T);
    int64_t* tasks = cv.take<int64_t>(T);
    int64_t* tsorted = cv.take<int64_t>(T);
    uint64_t* keys = cv.take<uint64_t>(T);
    uint64_t* keys2 = cv.take<uint64_t>(T);
    uint32_t* vals = cv.take<uint32_t>(T);
    uint32_t* vals2 = cv.take<uint32_t>(T);
    int64_t* hist = cv.take<int64_t>(hn);
    int64_t* htmp = cv.take<int64_t>(scan_tmp_elems(hn) + 64);
    if (!tasks || !tsorted || !keys || !keys2 || !vals || !vals2 || !hist || !htmp) return EBBKC_E_OOM;
    unsigned long long* cls_count = (unsigned long long*)(g->d_counters + 12);
    CHKH(hipMemsetAsync(cls_count, 0, 4 * sizeof(uint64_t), s));
    hipLaunchKernelGGL(k_task_fill, dim3(grid_for(n)), dim3(256), 0, s, g->seed_c, i0, n, l0, log_thr, toff, tasks,
                       keys, vals, cls_count);
    CHKH(radix_sort_u64(keys, vals, keys2, vals2, T, 10, hist, htmp, s));
    hipLaunchKernelGGL(k_gather_tasks, dim3(grid_for(T)), dim3(256), 0, s, tasks, vals, T, tsorted);
    CHKH(hipGetLastError());
    CHKH(hipMemcpyAsync(ccount, cls_count, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    *sorted = tsorted;
    return EBBKC_OK;
}

// scratch bytes for make_tasks over n slots with at most T tasks
static size_t task_bytes(int64_t n, int64_t T) {
    const int64_t hn = radix_hist_elems(T);
    return rnd256((size_t)n * 4) + rnd256((size_t)(n + 1) * 8) + rnd256((size_t)(scan_tmp_elems(n + 1) + 64) * 8) +
           4 * rnd256((size_t)T * 8) + 2 * rnd256((size_t)T * 4) + rnd256((size_t)hn * 8) +
           rnd256((size_t)(scan_tmp_elems(hn) + 64) * 8) + 4096;
}

// One search launch per width class over a sorted task list (classes are
// contiguous).  list = false: counts (per_task optional); list = true: tuples.
static ebbkc_status run_tasks(ebbkc_graph* g, int32_t k, const int64_t* tsorted, const uint64_t ccount[4],
                              uint64_t* per_task, const uint64_t* task_off, int32_t* out, void* gframes, bool list,
                              hipStream_t s, bool noalloc = false, SplitItem* squeue = nullptr,
                              unsigned long long* sq = nullptr) {
    // noalloc: no EBBkC-T rank slab and no timing events (the colour-ordered
    // search below the initial branch gives the same count under EBBkC-T)
    const bool truss = !list && !noalloc && g->opt.ordering == EBBKC_ORDER_TRUSS;
    if (truss) {  // EBBkC-T: depth limit and the per-wave rank matrices
        if (k > 2 * TRUSS_FRAMES + 3) return EBBKC_E_K_RANGE;
        if (!g->rho_slab) {
            hipError_t e = hipMalloc((void**)&g->rho_slab, truss_slab_bytes(g->cu_count));
            if (e != hipSuccess) {
                (void)hipGetLastError();
                g->rho_slab = nullptr;
                return e == hipErrorOutOfMemory ? EBBKC_E_OOM : EBBKC_E_HIP;
            }
        }
    }
    // listings up to k = 8 sort and hash each tuple as it is written
    unsigned long long* fused = list && k <= LIST_FUSED_K ? (unsigned long long*)(g->d_counters + 8) : nullptr;
    if (fused) CHKH(hipMemsetAsync(fused, 0, 2 * sizeof(uint64_t), s));
    hipEvent_t ev[MAX_W + 1][2] = {};
    int64_t off = 0;
    for (int W = 1; W <= MAX_W; ++W) {
        const int64_t nt = (int64_t)ccount[W - 1];
        if (!nt) continue;
        if (!noalloc) {
            CHKH(hipEventCreate(&ev[W][0]));
            CHKH(hipEventCreate(&ev[W][1]));
        }
        SearchArgs a{};
        a.A = ArenaView{g->seed_eid, g->seed_c, g->row_off, g->vtx_off, g->arows, g->agid, g->acol};
        a.tasks = tsorted + off;
        a.ntasks = nt;
        a.k = k;
        a.opts = opts_of(g->opt);
        a.k4_weight = k4_weight_of(g->opt.dense_k4);
        // under the vertex slots k is one above the clique size
        a.tplex = g->np_active && g->opt.t_plex == 0 ? (2 * (k - 1) <= g->tau ? 2 : 3) : g->opt.t_plex;
        a.tau = g->tau;
        a.next = (unsigned long long*)(g->d_counters + W - 1);
        a.total = (unsigned long long*)(g->d_counters + 4);
        a.work = (unsigned long long*)(g->d_counters + 16 + 4 * (W - 1));
        a.err = (int*)(g->d_counters + 6);
        a.per_task = per_task ? per_task + off : nullptr;
        a.task_off = task_off ? task_off + off : nullptr;
        a.out = out;
        a.eu = g->eu;
        a.ev = g->ev;
        a.list_checksums = fused;
        a.gframes = gframes;
        // runtime splitting: counts only (a queued node's count is not a task's own)
        if (squeue && !list && !truss && !per_task && g->opt.node_split != -1 && g->opt.blocks_per_cu != -1) {
            a.squeue = squeue;
            a.sq = sq;
            a.split_mode = g->opt.node_split == 1 ? SPLIT_FORCED : SPLIT_ON_DEMAND;
            a.split_bound = g->opt.node_split == 1 ? 0 : (g->opt.node_split >= 2 ? (uint64_t)g->opt.node_split : NODE_SPLIT_DEFAULT);
            CHKH(launch_sq_reset(sq, squeue, s));
        }
        if (g->opt.count_work && !list && !truss) a.wave_time = (unsigned long long*)(g->d_counters + 32 + 4 * (W - 1));
        CHKH(hipMemsetAsync(a.next, 0, sizeof(uint64_t), s));
        if (ev[W][0]) CHKH(hipEventRecord(ev[W][0], s));
        if (list) {
            CHKH(launch_list(W, a, g->cu_count, s));
        } else if (truss) {
            TrussArgs t{};
            t.A = a.A;
            t.tasks = a.tasks;
            t.ntasks = a.ntasks;
            t.k = k;
            t.opts = a.opts;
            t.tplex = g->opt.t_plex;
            t.rp = g->rp;
            t.ci = g->ci;
            t.erank = g->erank;
            t.rho = g->rho_slab;
            t.next = a.next;
            t.total = a.total;
            t.work = a.work;
            t.err = a.err;
            t.per_task = a.per_task;
            CHKH(launch_search_truss(W, t, g->cu_count, s));
        } else {
            CHKH(launch_search(W, false, a, g->cu_count, g->opt.blocks_per_cu, s));
            if (a.squeue)
                CHKH(hipMemcpyAsync(g->d_counters + 48 + W - 1, sq + SQ_PUSHED, sizeof(uint64_t),
                                    hipMemcpyDeviceToDevice, s));
        }
        if (ev[W][1]) CHKH(hipEventRecord(ev[W][1], s));
        off += nt;
    }
    CHKH(hipStreamSynchronize(s));
    for (int W = 1; W <= MAX_W; ++W) {
        if (!ev[W][0]) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[W][0], ev[W][1]) == hipSuccess && !list) g->last_ms[W - 1] = ms;
        (void)hipEventDestroy(ev[W][0]);
        (void)hipEventDestroy(ev[W][1]);
    }
    return EBBKC_OK;
}

// A count's scratch: the handle's buffer, grown on demand, or (fixed != null)
// a fixed buffer of cap bytes that is never grown: a count that needs more
// returns EBBKC_E_SCRATCH, and nothing is allocated.
struct ScratchSrc {
    void* fixed = nullptr;
    size_t cap = 0;
};

static Carve carve_for(ebbkc_graph* g, const ScratchSrc& src, size_t bytes) {
    if (src.fixed) return Carve{bytes <= src.cap ? (char*)src.fixed : nullptr, 0, src.cap};
    char* p = (char*)scratch_get(g, bytes);
    return Carve{p, 0, p ? g->scratch_bytes : 0};
}

static ebbkc_status count_core(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, uint64_t* out,
                               hipStream_t s, const ScratchSrc& src);

ebbkc_status count_impl(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, const int64_t* d_eids, int64_t ne,
                        uint64_t* d_per_seed, uint64_t* out, hipStream_t s) {
    (void)d_eids;
    (void)ne;
    (void)d_per_seed;
    return count_core(g, k, r_begin, r_end, out, s, ScratchSrc{});
}

static ebbkc_status count_core(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, uint64_t* out,
                               hipStream_t s, const ScratchSrc& src) {
    const bool noalloc = src.fixed != nullptr;
    const ebbkc_status e_space = noalloc ? EBBKC_E_SCRATCH : EBBKC_E_OOM;
    if (k < 3 || k > MAX_K) return EBBKC_E_K_RANGE;
    if (noalloc && (!g->arena_built || !g->d_counters || !g->subsize_ready)) return EBBKC_E_INVALID_ARG;
    if (!noalloc && g->opt.ordering == EBBKC_ORDER_DEGEN_VERTEX_NP && !g->np_active && r_begin <= 0 &&
        (r_end < 0 || r_end >= g->m) && k + 1 <= MAX_K) {
        // node-parallel VBBkC: one root per vertex v whose (k-1)-cliques in
        // G[N+(v)] are counted, i.e. the edge-slot search at k + 1 over the
        // vertex slots
        ebbkc_status st = vertex_arena_impl(g, s);
        if (st) return st;
        swap_arenas(g);
        st = count_core(g, k + 1, 0, -1, out, s, src);
        swap_arenas(g);
        return st;
    }
    ebbkc_status st = ensure_counters(g);  // allocated already under noalloc (checked above)
    if (st) return st;
    if (ensure_binom(g->device, s) != hipSuccess) return EBBKC_E_HIP;
    if (r_end < 0 || r_end > g->m) r_end = g->m;
    if (r_begin < 0) r_begin = 0;
    for (int i = 0; i < 4; ++i) g->last_ms[i] = 0.0;
    for (int i = 0; i < 4; ++i) g->last_work[i] = 0;
    for (int W = 0; W < 4; ++W)
        for (int i = 0; i < 4; ++i) g->last_work_class[W][i] = 0;
    CHKH(hipMemsetAsync(g->d_counters, 0, CNT_WORDS * sizeof(uint64_t), s));
    unsigned long long* total = (unsigned long long*)(g->d_counters + 4);
    if (k == 3) {  // sum of |V(g_i)| over the seeds
        st = subsize_impl(g, s);
        if (st) return st;
        if (r_end > r_begin)
            hipLaunchKernelGGL(k_sum_range, dim3(grid_for(r_end - r_begin)), dim3(256), 0, s, g->byrank, g->subsize,
                               (const uint64_t*)nullptr, r_begin, r_end, total);
        CHKH(hipGetLastError());
        return read_total(g, out, s);
    }
    st = arena_impl(g, s);
    if (st) return st;
    CHKH(hipMemsetAsync(g->d_counters, 0, CNT_WORDS * sizeof(uint64_t), s));
    const auto& SR = g->seed_rank_host;
    const int64_t i0 =
        std::lower_bound(SR.begin(), SR.end(), (int32_t)std::min<int64_t>(r_begin, INT32_MAX)) - SR.begin();
    const int64_t i1 =
        std::lower_bound(SR.begin(), SR.end(), (int32_t)std::min<int64_t>(r_end, INT32_MAX)) - SR.begin();
    const int64_t n = i1 - i0;
    if (k == 4) {  // sum of |E(g_i)| over the seeds
        if (n > 0)
            hipLaunchKernelGGL(k_sum_range, dim3(grid_for(n)), dim3(256), 0, s, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, g->nedges, i0, i1, total);
        CHKH(hipGetLastError());
        return read_total(g, out, s);
    }
    if (n <= 0) return read_total(g, out, s);
    const int l0 = k - 2;
    const double thr = g->opt.split_threshold > 0 ? (double)g->opt.split_threshold : (double)(1 << 22);
    const double log_thr = g->opt.split_threshold < 0 ? 1e300 : std::log(thr);

    // ---- tasks (the scratch is sized for the worst case: every slot split)
    const int64_t Tmax = n * (int64_t)(64 * MAX_W);
    const bool deep = k > SEARCH_DEEP_K;
    int64_t waves_max = 0;
    for (int W = 1; W <= MAX_W; ++W)
        waves_max = std::max(waves_max, search_grid_waves(W, false, Tmax, g->cu_count, g->opt.blocks_per_cu));
    const size_t fbytes = deep ? (size_t)waves_max * GLOBAL_FRAMES * search_frame_bytes(MAX_W) : 0;
    // count the real number of tasks first with a small scratch, then size
    Carve cv0 = carve_for(g, src, task_bytes(n, 1));
    int32_t* tcount = cv0.take<int32_t>(n);
    int64_t* toff = cv0.take<int64_t>(n + 1);
    int64_t* tmp = cv0.take<int64_t>(scan_tmp_elems(n + 1) + 64);
    if (!tcount || !toff || !tmp) return e_space;
    hipLaunchKernelGGL(k_task_counts, dim3(grid_for(n)), dim3(256), 0, s, g->seed_c, i0, n, l0, log_thr, tcount);
    CHKH(exclusive_scan_i32(tcount, toff, n, toff + n, tmp, s));
    int64_t T = 0;
    CHKH(hipMemcpyAsync(&T, toff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHKH(hipStreamSynchronize(s));
    if (T == 0) return read_total(g, out, s);
    const size_t qbytes = rnd256((size_t)SQ_CAP * sizeof(SplitItem)) + rnd256(SQ_WORDS * sizeof(uint64_t));
    Carve cv = carve_for(g, src, task_bytes(n, T) + rnd256(fbytes) + qbytes);
    if (!cv.base) return e_space;
    int64_t* tsorted = nullptr;
    uint64_t ccount[4] = {0, 0, 0, 0};
    int64_t T2 = 0;
    st = make_tasks(g, i0, n, l0, log_thr, s, cv, &tsorted, &T2, ccount);
    if (st) return st == EBBKC_E_OOM ? e_space : st;
    void* gframes = deep ? (void*)cv.take<char>((int64_t)fbytes) : nullptr;
    if (deep && !gframes) return e_space;
    SplitItem* squeue = cv.take<SplitItem>(SQ_CAP);
    unsigned long long* sq = cv.take<unsigned long long>(SQ_WORDS);
    if (!squeue || !sq) return e_space;

    // ---- search, one launch per width class
    st = run_tasks(g, k, tsorted, ccount, nullptr, nullptr, nullptr, gframes, false, s, noalloc, squeue, sq);
    if (st) return st;
    return read_total(g, out, s);
}

static int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b)) ++b;
    return b;
}

ebbkc_status list_impl(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, int32_t* d_buf, uint64_t cap,
                       uint32_t flags, uint64_t* out_written, uint64_t* out_checksums, hipStream_t s) {
    if (k < 1 || k > 64) return EBBKC_E_K_RANGE;
    ebbkc_status st = ensure_counters(g);
    if (st) return st;
    if (ensure_binom(g->device, s) != hipSuccess) return EBBKC_E_HIP;
    if (r_end < 0 || r_end > g->m) r_end = g->m;
    if (r_begin < 0 || r_begin > r_end) return EBBKC_E_INVALID_ARG;
    uint64_t N = 0;
    void* tmp_sort = nullptr;
    struct FreeOnExit { void*& p; ~FreeOnExit() { if (p) (void)hipFree(p); } } fe{tmp_sort};
    if (k <= 2) {
        if (k == 1 && (r_begin != 0 || r_end != g->m)) return EBBKC_E_INVALID_ARG;
        N = k == 1 ? (uint64_t)g->n : (uint64_t)(r_end - r_begin);
        *out_written = N;
        if (N > cap) return EBBKC_E_BUFFER_TOO_SMALL;
        if (N) CHKH(list_small(g->byrank, g->eu, g->ev, k == 1 ? 0 : r_begin, k == 1 ? g->n : r_end, k, d_buf, s));
    } else {
        st = arena_impl(g, s);
        if (st) return st;
        CHKH(hipMemsetAsync(g->d_counters, 0, CNT_WORDS * sizeof(uint64_t), s));
        const auto& SR = g->seed_rank_host;
        const int64_t i0 =
            std::lower_bound(SR.begin(), SR.end(), (int32_t)std::min<int64_t>(r_begin, INT32_MAX)) - SR.begin();
        const int64_t i1 =
            std::lower_bound(SR.begin(), SR.end(), (int32_t)std::min<int64_t>(r_end, INT32_MAX)) - SR.begin();
        const int64_t n = i1 - i0;
        if (n > 0) {
            const int l0 = k - 2;
            const double thr = g->opt.split_threshold > 0 ? (double)g->opt.split_threshold : (double)(1 << 22);
            const double log_thr = g->opt.split_threshold < 0 ? 1e300 : std::log(thr);
            Carve cv0{(char*)scratch_get(g, task_bytes(n, 1)), 0, 0};
            cv0.cap = g->scratch_bytes;
            int32_t* tcount = cv0.take<int32_t>(n);
            int64_t* toff = cv0.take<int64_t>(n + 1);
            int64_t* tmp = cv0.take<int64_t>(scan_tmp_elems(n + 1) + 64);
            if (!tcount || !toff || !tmp) return EBBKC_E_OOM;
            hipLaunchKernelGGL(k_task_counts, dim3(grid_for(n)), dim3(256), 0, s, g->seed_c, i0, n, l0, log_thr,
                               tcount);
            CHKH(exclusive_scan_i32(tcount, toff, n, toff + n, tmp, s));
            int64_t T = 0;
            CHKH(hipMemcpyAsync(&T, toff + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            CHKH(hipStreamSynchronize(s));
            if (T > 0) {
                // pass 1 runs the count kernel, pass 2 the listing kernel: frames
                // in device memory when either needs them
                const bool deep = k > std::min(SEARCH_DEEP_K, LIST_DEEP_K);
                const int64_t waves = list_grid_waves(MAX_W, T, g->cu_count);
                const int64_t wsearch = search_grid_waves(MAX_W, false, T, g->cu_count, g->opt.blocks_per_cu);
                const size_t fbytes = deep ? (size_t)std::max(waves, wsearch) * GLOBAL_FRAMES *
                                                 std::max(list_frame_bytes(MAX_W), search_frame_bytes(MAX_W))
                                           : 0;
                const size_t need = task_bytes(n, T) + rnd256(fbytes) + 2 * rnd256((size_t)(T + 1) * 8) +
                                    rnd256((size_t)(scan_tmp_elems(T + 1) + 64) * 8);
                if (!scratch_get(g, need)) return EBBKC_E_OOM;
                Carve cv{(char*)g->scratch, 0, g->scratch_bytes};
                int64_t* tsorted = nullptr;
                uint64_t ccount[4] = {0, 0, 0, 0};
                int64_t T2 = 0;
                st = make_tasks(g, i0, n, l0, log_thr, s, cv, &tsorted, &T2, ccount);
                if (st) return st;
                void* gframes = deep ? (void*)cv.take<char>((int64_t)fbytes) : nullptr;
                uint64_t* per_task = cv.take<uint64_t>(T + 1);
                uint64_t* task_off = cv.take<uint64_t>(T + 1);
                int64_t* stmp = cv.take<int64_t>(scan_tmp_elems(T + 1) + 64);
                if ((deep && !gframes) || !per_task || !task_off || !stmp) return EBBKC_E_OOM;
                // pass 1: per-task counts
                CHKH(hipMemsetAsync(g->d_counters + 4, 0, 4 * sizeof(uint64_t), s));
                st = run_tasks(g, k, tsorted, ccount, per_task, nullptr, nullptr, gframes, false, s);
                if (st) return st;
                st = read_total(g, &N, s);
                if (st) return st;
                *out_written = N;
                if (N > cap) return EBBKC_E_BUFFER_TOO_SMALL;
                CHKH(exclusive_scan_i64((const int64_t*)per_task, (int64_t*)task_off, T, nullptr, stmp, s));
                // pass 2: tuples
                st = run_tasks(g, k, tsorted, ccount, per_task, task_off, d_buf, gframes, true, s);
                if (st) return st;
                uint64_t herr = 0;
                CHKH(hipMemcpyAsync(&herr, g->d_counters + 6, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
                CHKH(hipStreamSynchronize(s));
                if (herr & ERR_CAP) return EBBKC_E_HIP;
                if (herr & ERR_DEPTH) return EBBKC_E_K_RANGE;
            }
        }
        *out_written = N;
    }
    // k_list wrote sorted tuples and their checksums (buffer order) for 3 <= k <= 8
    const bool fused = k >= 3 && k <= LIST_FUSED_K;
    const bool resorted = (flags & EBBKC_LIST_SORTED) && N > 1;
    if (N > 0) {
        if (!fused) CHKH(canon_tuples(d_buf, (int64_t)N, k, s));
        if (resorted) {
            const int bits = std::max(1, bits_for((uint64_t)(g->n > 0 ? g->n - 1 : 0)));
            const int64_t hn = radix_hist_elems((int64_t)N);
            const size_t bytes = 2 * rnd256(N * 8) + 2 * rnd256(N * 4) + rnd256((size_t)hn * 8) +
                                 rnd256((size_t)(scan_tmp_elems(hn) + 64) * 8) + rnd256(N * (size_t)k * 4) + 4096;
            CHKH(hipMalloc(&tmp_sort, bytes));
            Carve cv{(char*)tmp_sort, 0, bytes};
            uint64_t* keys = cv.take<uint64_t>((int64_t)N);
            uint64_t* keys2 = cv.take<uint64_t>((int64_t)N);
            uint32_t* idx = cv.take<uint32_t>((int64_t)N);
            uint32_t* idx2 = cv.take<uint32_t>((int64_t)N);
            int64_t* hist = cv.take<int64_t>(hn);
            int64_t* htmp = cv.take<int64_t>(scan_tmp_elems(hn) + 64);
            int32_t* tbuf = cv.take<int32_t>((int64_t)N * k);
            if (!keys || !keys2 || !idx || !idx2 || !hist || !htmp || !tbuf) return EBBKC_E_OOM;
            if (N >= ((uint64_t)1 << 32)) return EBBKC_E_INVALID_ARG;
            CHKH(sort_tuples(d_buf, (int64_t)N, k, bits, keys, keys2, idx, idx2, hist, htmp, tbuf, s));
        }
    }
    if (out_checksums) {
        if (fused && !resorted && N > 0) {
            CHKH(hipMemcpyAsync(out_checksums, g->d_counters + 8, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        } else {
            CHKH(tuple_checksums(d_buf, (int64_t)N, k, (unsigned long long*)(g->d_counters + 12), s));
            CHKH(hipMemcpyAsync(out_checksums, g->d_counters + 12, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        }
    }
    CHKH(hipStreamSynchronize(s));
    return EBBKC_OK;
}

// ---------------------------------------------------------------- count without allocation
// The fixed scratch of ebbkc_count_noalloc: task lists, sort buffers and deep
// search frames of one count.  Each device holds its own copy from the load
// of the library to the end of the process; host code reaches it only through
// the address hipGetSymbolAddress returns for that device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::once_flag g_scratch_once[NOALLOC_MAX_DEVICES];
void* g_scratch_ptr[NOALLOC_MAX_DEVICES];
hipError_t g_scratch_err[NOALLOC_MAX_DEVICES];

// device address of the fixed scratch on device dev, looked up once per
// device with that device current
void* noalloc_scratch(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
    std::call_once(g_scratch_once[dev], [dev] {
        int cur = 0;
        g_scratch_err[dev] = hipGetDevice(&cur);
        if (g_scratch_err[dev] != hipSuccess) return;
        if (cur != dev) g_scratch_err[dev] = hipSetDevice(dev);
        if (g_scratch_err[dev] == hipSuccess)
            g_scratch_err[dev] = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (g_scratch_err[dev] != hipSuccess) {
            (void)hipGetLastError();
            g_scratch_ptr[dev] = nullptr;
        }
    });
    return g_scratch_err[dev] == hipSuccess ? g_scratch_ptr[dev] : nullptr;
}
}  // namespace

ebbkc_status count_noalloc_impl(ebbkc_graph* g, int32_t k, uint64_t* out, hipStream_t s) {
    void* p = noalloc_scratch(g->device);
    if (!p) return EBBKC_E_HIP;
    return count_core(g, k, 0, g->m, out, s, ScratchSrc{p, NOALLOC_SCRATCH_BYTES});
}

// Per-seed counts for listed edge ids: one whole-root task per seed.
ebbkc_status count_seeds_impl(ebbkc_graph* g, int32_t k, const int64_t* eids, int64_t ne, int32_t ptr_kind,
                              uint64_t* out, hipStream_t s) {
    if (k < 3 || k > MAX_K) return EBBKC_E_K_RANGE;
    ebbkc_status st = ensure_counters(g);
    if (st) return st;
    if (ensure_binom(g->device, s) != hipSuccess) return EBBKC_E_HIP;
    st = arena_impl(g, s);
    if (st) return st;
    if (ne <= 0) return EBBKC_OK;
    std::vector<int64_t> he((size_t)ne);
    if (ptr_kind == EBBKC_PTR_DEVICE) CHKH(hipMemcpy(he.data(), eids, sizeof(int64_t) * ne, hipMemcpyDeviceToHost));
    else std::copy(eids, eids + ne, he.begin());
    if (g->seed_c_host.empty() && g->nseeds) {
        g->seed_c_host.resize((size_t)g->nseeds);
        CHKH(hipMemcpy(g->seed_c_host.data(), g->seed_c, sizeof(int32_t) * g->nseeds, hipMemcpyDeviceToHost));
    }
    if (g->rank_host.empty() && g->m) {
        g->rank_host.resize((size_t)g->m);
        CHKH(hipMemcpy(g->rank_host.data(), g->rank, sizeof(int32_t) * g->m, hipMemcpyDeviceToHost));
    }
    // tasks grouped by width class; task i -> output position
    std::vector<int64_t> tasks[MAX_W];
    std::vector<int64_t> where[MAX_W];
    std::vector<uint64_t> res((size_t)ne, 0);
    const auto& SR = g->seed_rank_host;
    for (int64_t i = 0; i < ne; ++i) {
        const int64_t e = he[(size_t)i];
        if (e < 0 || e >= g->m) return EBBKC_E_INVALID_ARG;
        const int32_t r = g->rank_host[(size_t)e];
        const int64_t slot = std::lower_bound(SR.begin(), SR.end(), r) - SR.begin();
        if (slot >= (int64_t)SR.size() || SR[(size_t)slot] != r) continue;  // empty sub-branch
        const int c = g->seed_c_host[(size_t)slot];
        if (c < k - 2) continue;
        tasks[width_of(c) - 1].push_back(task_pack(slot, 0, c));
        where[width_of(c) - 1].push_back(i);
    }
    uint64_t ccount[4];
    int64_t T = 0;
    for (int W = 0; W < MAX_W; ++W) { ccount[W] = tasks[W].size(); T += (int64_t)tasks[W].size(); }
    if (T) {
        const bool deep = k > SEARCH_DEEP_K;
        const size_t fbytes =
            deep ? (size_t)search_grid_waves(MAX_W, false, T, g->cu_count, g->opt.blocks_per_cu) * GLOBAL_FRAMES *
                       search_frame_bytes(MAX_W)
                 : 0;
        if (!scratch_get(g, rnd256(T * 8) * 2 + rnd256(fbytes) + 4096)) return EBBKC_E_OOM;
        Carve cv{(char*)g->scratch, 0, g->scratch_bytes};
        int64_t* dt = cv.take<int64_t>(T);
        uint64_t* pt = cv.take<uint64_t>(T);
        void* gframes = deep ? (void*)cv.take<char>((int64_t)fbytes) : nullptr;
        std::vector<int64_t> flat;
        flat.reserve((size_t)T);
        for (int W = 0; W < MAX_W; ++W) flat.insert(flat.end(), tasks[W].begin(), tasks[W].end());
        CHKH(hipMemcpyAsync(dt, flat.data(), sizeof(int64_t) * T, hipMemcpyHostToDevice, s));
        CHKH(hipMemsetAsync(g->d_counters, 0, CNT_WORDS * sizeof(uint64_t), s));
        st = run_tasks(g, k, dt, ccount, pt, nullptr, nullptr, gframes, false, s);
        if (st) return st;
        uint64_t tot = 0;
        st = read_total(g, &tot, s);
        if (st) return st;
        std::vector<uint64_t> hp((size_t)T);
        CHKH(hipMemcpy(hp.data(), pt, sizeof(uint64_t) * T, hipMemcpyDeviceToHost));
        int64_t o = 0;
        for (int W = 0; W < MAX_W; ++W)
            for (size_t j = 0; j < where[W].size(); ++j) res[(size_t)where[W][j]] = hp[(size_t)o++];
    }
    if (ptr_kind == EBBKC_PTR_DEVICE) CHKH(hipMemcpy(out, res.data(), sizeof(uint64_t) * ne, hipMemcpyHostToDevice));
    else std::copy(res.begin(), res.end(), out);
    return EBBKC_OK;
}

}  // namespace ebb
