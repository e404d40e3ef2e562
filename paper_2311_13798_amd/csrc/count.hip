// count.hip -- host orchestration of the branch kernels: seed selection by
// rank range and width class, persistent launches, exact 128-bit totals.
//
// Seeds.  A sub-branch of seed e_i has at most level(e_i) vertices (the peel
// removes e_i with at most that many common neighbours among later edges), so
// for a given k only edges with level >= k-2 can hold a k-clique.  Levels are
// non-decreasing along the ranking, hence those seeds are one suffix of the
// rank order, and each bitmap width class (64, 128, 192, 256 vertices) is a
// contiguous rank interval inside it.  Classes are launched widest first and
// each kernel hands out its seeds from the highest rank down (heaviest
// first).
#include <algorithm>
#include <mutex>

#include "branch.h"
#include "common.h"
#include "handle.h"

namespace ebb {

constexpr int MAX_W = 4;

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
    if (o.t_plex >= 2) f |= OPT_TPLEX2;
    if (o.rule1) f |= OPT_RULE1;
    if (o.rule2) f |= OPT_RULE2;
    if (o.count_work) f |= OPT_WORK;
    return f;
}

// counters block: [0..MAX_W) seed counters per class, [4,5] total lo/hi,
// [6] error flags, [8..10] search work
constexpr int CNT_WORDS = 12;

}  // namespace

void* scratch_get(ebbkc_graph* g, size_t bytes) {
    if (bytes <= g->scratch_bytes) return g->scratch;
    if (g->scratch) (void)hipFree(g->scratch);
    g->scratch = nullptr;
    g->scratch_bytes = 0;
    size_t nb = bytes + bytes / 4;
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

static BranchArgs base_args(ebbkc_graph* g, int32_t k) {
    BranchArgs a{};
    a.rp = g->rp;
    a.ci = g->ci;
    a.erank = g->erank;
    a.rrow = g->rrow;
    a.orp = g->orp;
    a.orow = g->orow;
    a.eu = g->eu;
    a.ev = g->ev;
    a.rank = g->rank;
    a.k = k;
    a.opts = opts_of(g->opt);
    a.total = (unsigned long long*)(g->d_counters + 4);
    a.err = (int*)(g->d_counters + 6);
    a.work = (unsigned long long*)(g->d_counters + 8);
    return a;
}

static ebbkc_status finish_total(ebbkc_graph* g, uint64_t* out, hipStream_t s) {
    if (hipMemcpyAsync(g->h_counters, g->d_counters, CNT_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, s) !=
        hipSuccess)
        return EBBKC_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return EBBKC_E_HIP;
    int err = (int)g->h_counters[6];
    if (err & ERR_WIDTH) return EBBKC_E_WIDTH;
    if (err & ERR_DEPTH) return EBBKC_E_K_RANGE;
    if ((err & ERR_OVERFLOW) || g->h_counters[5] != 0) return EBBKC_E_OVERFLOW;
    *out = g->h_counters[4];
    for (int i = 0; i < 3; ++i) g->last_work[i] = g->h_counters[8 + i];
    return EBBKC_OK;
}

// Rank interval [lo, hi) of seeds able to hold a k-clique, split by width
// class; cls[W] = [lo_W, hi_W).
static ebbkc_status class_ranges(const ebbkc_graph* g, int32_t k, int64_t lo, int64_t hi, int64_t cls[MAX_W + 1][2]) {
    const auto& L = g->lvl_by_rank;
    int64_t first = std::lower_bound(L.begin(), L.end(), k - 2) - L.begin();
    if (lo < first) lo = first;
    for (int W = 0; W <= MAX_W; ++W) cls[W][0] = cls[W][1] = 0;
    if (lo >= hi) return EBBKC_OK;
    if (L[(size_t)hi - 1] > 64 * MAX_W) return EBBKC_E_WIDTH;
    for (int W = 1; W <= MAX_W; ++W) {
        int64_t a = W == 1 ? 0 : std::lower_bound(L.begin(), L.end(), 64 * (W - 1) + 1) - L.begin();
        int64_t b = std::lower_bound(L.begin(), L.end(), 64 * W + 1) - L.begin();
        a = std::max(a, lo);
        b = std::min(b, hi);
        if (b > a) { cls[W][0] = a; cls[W][1] = b; }
    }
    return EBBKC_OK;
}

ebbkc_status count_impl(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, const int64_t* d_eids, int64_t ne,
                        uint64_t* d_per_seed, uint64_t* out, hipStream_t s) {
    (void)d_eids;
    (void)ne;
    if (k < 1) return EBBKC_E_K_RANGE;
    if (k > MAX_K) return EBBKC_E_K_RANGE;
    ebbkc_status st = ensure_counters(g);
    if (st) return st;
    if (ensure_binom(g->device, s) != hipSuccess) return EBBKC_E_HIP;
    if (r_end < 0 || r_end > g->m) r_end = g->m;
    if (r_begin < 0) r_begin = 0;
    if (hipMemsetAsync(g->d_counters, 0, CNT_WORDS * sizeof(uint64_t), s) != hipSuccess) return EBBKC_E_HIP;
    if (d_per_seed && r_end > r_begin)
        if (hipMemsetAsync(d_per_seed, 0, sizeof(uint64_t) * (size_t)(r_end - r_begin), s) != hipSuccess)
            return EBBKC_E_HIP;
    int64_t cls[MAX_W + 1][2];
    st = class_ranges(g, k, r_begin, r_end, cls);
    if (st) return st;
    // deep searches need frames in device memory: one allocation for all classes
    void* gframes = nullptr;
    if (k > 2 + 2 * MAX_FRAMES + 2) {
        size_t need = 0;
        for (int W = 1; W <= MAX_W; ++W) {
            if (cls[W][1] <= cls[W][0]) continue;
            int64_t waves = branch_grid_waves(W, cls[W][1] - cls[W][0], g->cu_count, g->opt.blocks_per_cu);
            if (waves < 0) return EBBKC_E_HIP;
            need = std::max(need, (size_t)waves * GLOBAL_FRAMES * branch_frame_bytes(W));
        }
        if (need) {
            gframes = scratch_get(g, need);
            if (!gframes) return EBBKC_E_OOM;
        }
    }
    hipEvent_t ev[MAX_W + 1][2] = {};
    for (int W = 1; W <= MAX_W; ++W) {
        g->last_ms[W - 1] = 0.0;
        if (cls[W][1] <= cls[W][0]) continue;
        if (hipEventCreate(&ev[W][0]) != hipSuccess || hipEventCreate(&ev[W][1]) != hipSuccess) return EBBKC_E_HIP;
    }
    for (int W = MAX_W; W >= 1; --W) {
        int64_t a0 = cls[W][0], a1 = cls[W][1];
        if (a1 <= a0) continue;
        BranchArgs a = base_args(g, k);
        a.gframes = gframes;
        a.seeds = g->byrank + a0;
        a.nseeds = a1 - a0;
        a.reverse = 1;
        a.out_base = a0 - r_begin;
        a.per_seed = d_per_seed;
        a.next = (unsigned long long*)(g->d_counters + (W - 1));
        (void)hipEventRecord(ev[W][0], s);
        if (launch_branch_class(W, false, a, g->cu_count, g->opt.blocks_per_cu, s) != hipSuccess) return EBBKC_E_HIP;
        (void)hipEventRecord(ev[W][1], s);
    }
    st = finish_total(g, out, s);
    for (int W = 1; W <= MAX_W; ++W) {
        if (!ev[W][0]) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[W][0], ev[W][1]) == hipSuccess) g->last_ms[W - 1] = ms;
        (void)hipEventDestroy(ev[W][0]);
        (void)hipEventDestroy(ev[W][1]);
    }
    return st;
}

ebbkc_status subsize_impl(ebbkc_graph* g, hipStream_t s) {
    if (g->subsize_ready) return EBBKC_OK;
    if (!g->subsize && hipMalloc((void**)&g->subsize, sizeof(int32_t) * (size_t)(g->m > 0 ? g->m : 1)) != hipSuccess)
        return EBBKC_E_OOM;
    if (launch_subsize(g->rp, g->ci, g->erank, g->rrow, g->eu, g->ev, g->rank, g->m, g->subsize, s) != hipSuccess)
        return EBBKC_E_HIP;
    g->subsize_ready = true;
    return EBBKC_OK;
}

}  // namespace ebb
