// prepare.hip -- CSR intake, edge supports and the level-synchronous
// truss-based edge ordering (Section 4.2 of the paper, Eq. truss-based-edge),
// then the rank-tagged adjacency the branching kernels read.
//
// Pipeline (all on the device, one stream):
//   validate   rows strictly ascending, ids in range, no self-loops, symmetric
//   edge ids   edge (u,v), u<v, gets its rank in lexicographic order
//   triangles  degree orientation (a->b iff (deg a, a) < (deg b, b)); every
//              triangle is found once from its first oriented edge, counted
//              into the three edges' supports, then written as "the other two
//              edges" into each edge's incidence list
//   peel       level s, round r: every remaining edge with support <= s forms
//              the frontier; frontier edges get level s and rank (round, id);
//              each triangle destroyed in the round lowers each surviving edge
//              once (its lowest-id frontier edge does it); when no edge
//              qualifies s jumps to the smallest remaining support
//   adjacency  erank (rank of each CSR entry), rows re-sorted by rank
//              descending, and degree-oriented rows in the same order
#include <chrono>
#include <vector>

#include "arena.h"
#include "common.h"
#include "device_util.h"
#include "handle.h"
#include "prims.h"

namespace ebb {
namespace {

constexpr int TB = 256;

inline unsigned grid_for(int64_t n, int per = TB) {
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > 65535 * 32) b = 65535 * 32;
    return (unsigned)b;
}

// row of CSR entry p (rp must be monotone; garbage otherwise, caught by validation)
__device__ __forceinline__ int32_t row_of(const int32_t* __restrict__ rp, int32_t n, int64_t p) {
    int lo = 0, hi = n;  // find largest u with rp[u] <= p
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_validate_rows(const int32_t* __restrict__ rp, int32_t n, int64_t nnz, int* __restrict__ err) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    if (u == 0 && rp[0] != 0) atomicOr(err, 1);
    if (u == n && (int64_t)rp[n] != nnz) atomicOr(err, 2);
    if (u < n && rp[u + 1] < rp[u]) atomicOr(err, 4);
}

__global__ void k_validate_entries(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int32_t n,
                                   int64_t nnz, int* __restrict__ err) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = row_of(rp, n, p);
        int32_t v = ci[p];
        if (v < 0 || v >= n || v == u) { atomicOr(err, 8); continue; }
        if (p > rp[u] && ci[p - 1] >= v) { atomicOr(err, 16); continue; }
        int q = lower_bound_i32(ci, rp[v], rp[v + 1], u);
        if (q >= rp[v + 1] || ci[q] != u) atomicOr(err, 32);
    }
}

// ustart[u] = first entry of row u with neighbour > u; ucnt[u] = entries after it; degree max
__global__ void k_ustart(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int32_t n,
                         int32_t* __restrict__ ustart, int32_t* __restrict__ ucnt, int* __restrict__ dmax) {
    int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int q = lower_bound_i32(ci, rp[u], rp[u + 1], u + 1);
    ustart[u] = q;
    ucnt[u] = rp[u + 1] - q;
    atomicMax(dmax, rp[u + 1] - rp[u]);
}

__global__ void k_edge_ids(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int32_t n, int64_t nnz,
                           const int32_t* __restrict__ ustart, const int64_t* __restrict__ eoff,
                           int32_t* __restrict__ eid, int32_t* __restrict__ src, int32_t* __restrict__ eu,
                           int32_t* __restrict__ ev) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        int32_t u = row_of(rp, n, p);
        int32_t v = ci[p];
        int64_t e;
        if (v > u) {
            e = eoff[u] + (p - ustart[u]);
            eu[e] = u;
            ev[e] = v;
        } else {
            int q = lower_bound_i32(ci, ustart[v], rp[v + 1], u);
            e = eoff[v] + (q - ustart[v]);
        }
        eid[p] = (int32_t)e;
        src[p] = u;
    }
}

__device__ __forceinline__ bool oriented_before(int32_t a, int32_t da, int32_t b, int32_t db) {
    return da < db || (da == db && a < b);
}

// out-degree of every vertex under the degree orientation
__global__ void k_out_count(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int32_t n,
                            int32_t* __restrict__ ocnt) {
    int wid = (blockIdx.x * blockDim.x + threadIdx.x) / EBB_WAVE;
    int nw = gridDim.x * blockDim.x / EBB_WAVE;
    for (int32_t a = wid; a < n; a += nw) {
        int32_t da = rp[a + 1] - rp[a], c = 0;
        for (int32_t p = rp[a] + lane_id(); p < rp[a + 1]; p += EBB_WAVE) {
            int32_t b = ci[p];
            c += oriented_before(a, da, b, rp[b + 1] - rp[b]);
        }
        c = wave_sum(c);
        if (lane_id() == 0) ocnt[a] = c;
    }
}

// Ordered compaction of each row's out-entries.  mode 0: id-sorted rows
// (col, eid); mode 1: rank-sorted rows (col, rank) taken from rrow.
__global__ void k_out_fill(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const int32_t* __restrict__ eid, const int2* __restrict__ rrow, int32_t n,
                           const int64_t* __restrict__ ooff, int2* __restrict__ out, int32_t* __restrict__ osrc,
                           int mode) {
    int wid = (blockIdx.x * blockDim.x + threadIdx.x) / EBB_WAVE;
    int nw = gridDim.x * blockDim.x / EBB_WAVE;
    for (int32_t a = wid; a < n; a += nw) {
        int32_t da = rp[a + 1] - rp[a];
        int64_t w = ooff[a];
        for (int32_t base = rp[a]; base < rp[a + 1]; base += EBB_WAVE) {
            int32_t p = base + lane_id();
            bool in = p < rp[a + 1];
            int2 val = make_int2(0, 0);
            bool keep = false;
            if (in) {
                int32_t b = mode == 0 ? ci[p] : rrow[p].x;
                keep = oriented_before(a, da, b, rp[b + 1] - rp[b]);
                val = mode == 0 ? make_int2(b, eid[p]) : rrow[p];
            }
            uint64_t mask = ballot(keep);
            if (keep) {
                int64_t q = w + popc64(mask & lanemask_lt());
                out[q] = val;
                if (osrc) osrc[q] = a;
            }
            w += popc64(mask);
        }
    }
}

// Triangles a->b, a->w, b->w found from oriented entry (a->b) by looking up
// each w of out(b) in out(a).  pass 0: count into sup; pass 1: write the
// incidence pairs.
__global__ void k_triangles(const int64_t* __restrict__ ooff, const int2* __restrict__ orow_id,
                            const int32_t* __restrict__ osrc, int64_t mo, int32_t* __restrict__ sup,
                            int64_t* __restrict__ cursor, int2* __restrict__ inc, int pass) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < mo; q += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = osrc[q];
        int2 ab = orow_id[q];
        int32_t b = ab.x, e_ab = ab.y;
        int64_t a0 = ooff[a], a1 = ooff[a + 1];
        for (int64_t t = ooff[b]; t < ooff[b + 1]; ++t) {
            int2 bw = orow_id[t];
            // binary search bw.x in out(a) (id-sorted)
            int64_t lo = a0, hi = a1;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (orow_id[mid].x < bw.x) lo = mid + 1; else hi = mid;
            }
            if (lo < a1 && orow_id[lo].x == bw.x) {
                int32_t e_aw = orow_id[lo].y, e_bw = bw.y;
                if (pass == 0) {
                    atomicAdd(&sup[e_ab], 1);
                    atomicAdd(&sup[e_aw], 1);
                    atomicAdd(&sup[e_bw], 1);
                } else {
                    inc[atomicAdd((unsigned long long*)&cursor[e_ab], 1ull)] = make_int2(e_aw, e_bw);
                    inc[atomicAdd((unsigned long long*)&cursor[e_aw], 1ull)] = make_int2(e_ab, e_bw);
                    inc[atomicAdd((unsigned long long*)&cursor[e_bw], 1ull)] = make_int2(e_ab, e_aw);
                }
            }
        }
    }
}

__global__ void k_iota(int32_t* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (int32_t)i;
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

struct PeelState {
    int32_t minsup;
    int32_t pad;
    int64_t nf;
};

__global__ void k_peel_reset(PeelState* st) {
    st->minsup = 0x7fffffff;
    st->nf = 0;
}

__global__ void k_peel_flag(const int32_t* __restrict__ live, int64_t nlive, const int32_t* __restrict__ sup,
                            int32_t s, int32_t* __restrict__ flag, PeelState* __restrict__ st) {
    int32_t mn = 0x7fffffff;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nlive; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t x = sup[live[i]];
        flag[i] = x <= s;
        mn = x < mn ? x : mn;
    }
    // one atomic per block
    __shared__ int32_t bm[TB / EBB_WAVE];
    mn = wave_min(mn);
    if (lane_id() == 0) bm[threadIdx.x / EBB_WAVE] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < TB / EBB_WAVE; ++i) mn = bm[i] < mn ? bm[i] : mn;
        mn = bm[0] < mn ? bm[0] : mn;
        if (mn < 0x7fffffff) atomicMin(&st->minsup, mn);
    }
}

__global__ void k_peel_compact(const int32_t* __restrict__ live, int64_t nlive, const int32_t* __restrict__ flag,
                               const int64_t* __restrict__ pos, int32_t* __restrict__ front,
                               int32_t* __restrict__ keep) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nlive; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t e = live[i];
        if (flag[i]) front[pos[i]] = e;
        else keep[i - pos[i]] = e;
    }
}

__global__ void k_peel_assign(const int32_t* __restrict__ front, int64_t nf, int32_t s, int64_t ranked, int32_t r,
                              int32_t* __restrict__ level, int32_t* __restrict__ rank, int32_t* __restrict__ rnd) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t e = front[i];
        level[e] = s;
        rank[e] = (int32_t)(ranked + i);
        rnd[e] = r;
    }
}

// one wave per frontier edge, lanes over its incident triangles
__global__ void k_peel_triangles(const int32_t* __restrict__ front, int64_t nf, const int64_t* __restrict__ inc_off,
                                 const int2* __restrict__ inc, const int32_t* __restrict__ rnd, int32_t r,
                                 int32_t* __restrict__ sup) {
    int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / EBB_WAVE;
    int64_t nw = (int64_t)gridDim.x * blockDim.x / EBB_WAVE;
    for (int64_t i = wid; i < nf; i += nw) {
        int32_t e = front[i];
        for (int64_t t = inc_off[e] + lane_id(); t < inc_off[e + 1]; t += EBB_WAVE) {
            int2 fg = inc[t];
            int32_t rf = rnd[fg.x], rg = rnd[fg.y];
            bool pf = rf < 0 || rf == r, pg = rg < 0 || rg == r;
            if (!(pf && pg)) continue;  // destroyed in an earlier round
            int32_t mine = e;
            if (rf == r && fg.x < mine) mine = fg.x;
            if (rg == r && fg.y < mine) mine = fg.y;
            if (mine != e) continue;
            if (rf < 0) atomicSub(&sup[fg.x], 1);
            if (rg < 0) atomicSub(&sup[fg.y], 1);
        }
    }
}

__global__ void k_erank_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ eid,
                             const int32_t* __restrict__ rank, int64_t nnz, int64_t m, int32_t* __restrict__ erank,
                             uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = rank[eid[p]];
        erank[p] = r;
        keys[p] = (uint64_t)src[p] * (uint64_t)m + (uint64_t)(m - 1 - r);
        vals[p] = (uint32_t)p;
    }
}

__global__ void k_gather_rrow(const uint32_t* __restrict__ perm, const int32_t* __restrict__ ci,
                              const int32_t* __restrict__ erank, int64_t nnz, int2* __restrict__ rrow) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t p = perm[i];
        rrow[i] = make_int2(ci[p], erank[p]);
    }
}

__global__ void k_byrank(const int32_t* __restrict__ rank, int64_t m, int32_t* __restrict__ byrank) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        byrank[rank[e]] = (int32_t)e;
}

// adjacency bitmap: one bit per CSR entry (a row's entries may share a word)
__global__ void k_adj_fill(const int32_t* __restrict__ src, const int32_t* __restrict__ ci, int64_t nnz, int32_t aw,
                           uint64_t* __restrict__ adj) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t w = ci[i];
        atomicOr((unsigned long long*)&adj[(int64_t)src[i] * aw + (w >> 6)], 1ull << (w & 63));
    }
}

// acum[x aw + q] = entries of x's id-sorted row below vertex 64 q
__global__ void k_adj_cum(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int32_t n, int32_t aw,
                          uint16_t* __restrict__ acum) {
    const int64_t total = (int64_t)n * aw;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = (int32_t)(t / aw), q = (int32_t)(t % aw);
        int lo = rp[x], hi = rp[x + 1];
        const int base = lo;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ci[mid] < 64 * q) lo = mid + 1; else hi = mid;
        }
        acum[t] = (uint16_t)(lo - base);
    }
}

// ---- vertex orders for the root edge order of the ablation orderings

// Greedy colouring in the visiting order (degree desc, id asc), one wave per
// vertex: a vertex takes the least colour >= 1 not held by its neighbours
// earlier in that order once all of them are coloured, which is the colour
// the sequential greedy pass gives it (Jones-Plassmann rounds).  A vertex
// still waiting adds one to *pending.
constexpr int CWIN = 4096;  // colours tested per window

__device__ __forceinline__ bool visits_before(int32_t w, int32_t dw, int32_t v, int32_t dv) {
    return dw > dv || (dw == dv && w < v);
}

__global__ __launch_bounds__(TB) void k_colour_round(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                     int32_t n, int32_t* col, int32_t* __restrict__ pending) {
    __shared__ uint32_t used[TB / EBB_WAVE][CWIN / 32];
    const int lane = lane_id(), wv = threadIdx.x / EBB_WAVE;
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / EBB_WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / EBB_WAVE;
    const volatile int32_t* vcol = col;
    int waiting = 0;
    for (int64_t vv = wid; vv < n; vv += nw) {
        const int32_t v = (int32_t)vv;
        if (__builtin_amdgcn_readfirstlane(vcol[v]) != 0) continue;
        const int32_t b = rp[v], e = rp[v + 1], dv = e - b;
        bool wait = false;
        for (int32_t j = b + lane; j < e; j += EBB_WAVE) {
            const int32_t w = ci[j];
            if (visits_before(w, rp[w + 1] - rp[w], v, dv) && vcol[w] == 0) wait = true;
        }
        if (ballot(wait)) { ++waiting; continue; }
        // the least colour absent from the earlier neighbours (at most dv of them)
        for (int32_t base = 1;; base += CWIN) {
            for (int i = lane; i < CWIN / 32; i += EBB_WAVE) used[wv][i] = 0;
            wave_sync();
            for (int32_t j = b + lane; j < e; j += EBB_WAVE) {
                const int32_t w = ci[j];
                if (!visits_before(w, rp[w + 1] - rp[w], v, dv)) continue;
                const int32_t cw = vcol[w] - base;
                if (cw >= 0 && cw < CWIN) atomicOr(&used[wv][cw >> 5], 1u << (cw & 31));
            }
            wave_sync();
            int first = CWIN;
            for (int i = lane; i < CWIN / 32; i += EBB_WAVE) {
                const uint32_t f = ~used[wv][i];
                if (f) { first = i * 32 + __builtin_ctz(f); break; }
            }
            first = wave_min(first);
            wave_sync();
            if (first < CWIN) {
                if (lane == 0) col[v] = base + first;
                break;
            }
        }
    }
    if (lane == 0 && waiting) atomicAdd(pending, waiting);
}

// colour order: key (colour desc), vertex id as the value; a stable sort keeps ids ascending
__global__ void k_colour_keys(const int32_t* __restrict__ col, int32_t n, uint64_t* __restrict__ keys,
                              uint32_t* __restrict__ vals) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        keys[v] = (uint64_t)(0x7fffffff - col[v]);
        vals[v] = (uint32_t)v;
    }
}

__global__ void k_scatter_pos(const uint32_t* __restrict__ vals, int64_t n, int32_t* __restrict__ pos) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        pos[vals[i]] = (int32_t)i;
}

__global__ void k_degrees(const int32_t* __restrict__ rp, int32_t n, int32_t* __restrict__ deg) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        deg[v] = rp[v + 1] - rp[v];
}

__global__ void k_core_assign(const int32_t* __restrict__ front, int64_t nf, int64_t placed, int32_t r,
                              int32_t* __restrict__ pos, int32_t* __restrict__ rnd) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += (int64_t)gridDim.x * blockDim.x) {
        pos[front[i]] = (int32_t)(placed + i);
        rnd[front[i]] = r;
    }
}

// one wave per removed vertex: its neighbours still present lose one degree
__global__ void k_core_remove(const int32_t* __restrict__ front, int64_t nf, const int32_t* __restrict__ rp,
                              const int32_t* __restrict__ ci, const int32_t* __restrict__ rnd,
                              int32_t* __restrict__ deg) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / EBB_WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / EBB_WAVE;
    for (int64_t i = wid; i < nf; i += nw) {
        const int32_t v = front[i];
        for (int32_t j = rp[v] + lane_id(); j < rp[v + 1]; j += EBB_WAVE) {
            const int32_t w = ci[j];
            if (rnd[w] < 0) atomicSub(&deg[w], 1);
        }
    }
}

// edge e = (u, v): key (min pos, max pos), lexicographic
__global__ void k_lex_edge_keys(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                                const int32_t* __restrict__ pos, int64_t m, int32_t n, uint64_t* __restrict__ keys,
                                uint32_t* __restrict__ vals) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = pos[eu[e]], b = pos[ev[e]];
        keys[e] = (uint64_t)(a < b ? a : b) * (uint64_t)n + (uint64_t)(a < b ? b : a);
        vals[e] = (uint32_t)e;
    }
}

__global__ void k_copy_i64_to_i32(const int64_t* __restrict__ a, int32_t* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (int32_t)a[i];
}

template <typename T>
struct DBuf {
    T* p = nullptr;
    hipError_t alloc(int64_t n) { return hipMalloc((void**)&p, sizeof(T) * (size_t)(n > 0 ? n : 1)); }
    ~DBuf() { if (p) (void)hipFree(p); }
    T* release() { T* q = p; p = nullptr; return q; }
};

int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b)) ++b;
    return b;
}

}  // namespace

#define CHK(expr)                                   \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) {                     \
            (void)hipGetLastError();                \
            return e_ == hipErrorOutOfMemory ? EBBKC_E_OOM : EBBKC_E_HIP; \
        }                                           \
    } while (0)

ebbkc_status prepare_impl(ebbkc_graph* g, const int32_t* row_ptr, const int32_t* col_idx, int32_t ptr_kind,
                          hipStream_t s) {
    const int32_t n = g->n;
    const int64_t nnz = g->nnz;
    hipEvent_t ev0, ev1;
    CHK(hipEventCreate(&ev0));
    CHK(hipEventCreate(&ev1));
    CHK(hipEventRecord(ev0, s));

    DBuf<int32_t> rp, ci;
    CHK(rp.alloc(n + 1));
    CHK(ci.alloc(nnz));
    hipMemcpyKind kind = ptr_kind == EBBKC_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    CHK(hipMemcpyAsync(rp.p, row_ptr, sizeof(int32_t) * (size_t)(n + 1), kind, s));
    if (nnz) CHK(hipMemcpyAsync(ci.p, col_idx, sizeof(int32_t) * (size_t)nnz, kind, s));

    // small host-visible status block: [0] err, [1] dmax
    int* hstat = nullptr;
    int* dstat = nullptr;
    CHK(hipHostMalloc((void**)&hstat, 4 * sizeof(int), hipHostMallocDefault));
    struct HostFree { int* p; ~HostFree() { if (p) (void)hipHostFree(p); } } hf{hstat};
    DBuf<int> stat;
    CHK(stat.alloc(4));
    dstat = stat.p;
    CHK(hipMemsetAsync(dstat, 0, 4 * sizeof(int), s));
    // row offsets first: the entry checks index rows through them
    hipLaunchKernelGGL(k_validate_rows, dim3(grid_for(n + 1)), dim3(TB), 0, s, rp.p, n, nnz, dstat);
    CHK(hipGetLastError());
    CHK(hipMemcpyAsync(hstat, dstat, sizeof(int), hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    if (hstat[0] != 0) return EBBKC_E_BAD_CSR;
    if (nnz) hipLaunchKernelGGL(k_validate_entries, dim3(grid_for(nnz)), dim3(TB), 0, s, rp.p, ci.p, n, nnz, dstat);
    CHK(hipGetLastError());
    CHK(hipMemcpyAsync(hstat, dstat, sizeof(int), hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    if (hstat[0] != 0) return EBBKC_E_BAD_CSR;
    if (nnz % 2 != 0) return EBBKC_E_BAD_CSR;
    const int64_t m = nnz / 2;
    g->m = m;

    // ---- edge ids
    DBuf<int32_t> ustart, ucnt, eid, src, eu, ev;
    DBuf<int64_t> eoff, scan_tmp;
    CHK(ustart.alloc(n));
    CHK(ucnt.alloc(n));
    CHK(eoff.alloc(n + 1));
    int64_t tmp_elems = scan_tmp_elems(nnz + n + 2) + 1024;
    CHK(scan_tmp.alloc(tmp_elems));
    CHK(eid.alloc(nnz));
    CHK(src.alloc(nnz));
    CHK(eu.alloc(m));
    CHK(ev.alloc(m));
    if (n) hipLaunchKernelGGL(k_ustart, dim3(grid_for(n)), dim3(TB), 0, s, rp.p, ci.p, n, ustart.p, ucnt.p, dstat + 1);
    CHK(exclusive_scan_i32(ucnt.p, eoff.p, n, eoff.p + n, scan_tmp.p, s));
    if (nnz)
        hipLaunchKernelGGL(k_edge_ids, dim3(grid_for(nnz)), dim3(TB), 0, s, rp.p, ci.p, n, nnz, ustart.p, eoff.p,
                           eid.p, src.p, eu.p, ev.p);
    CHK(hipGetLastError());

    // ---- degree orientation (id-sorted out rows with edge ids)
    DBuf<int32_t> ocnt, osrc;
    DBuf<int64_t> ooff;
    DBuf<int2> orow_id;
    CHK(ocnt.alloc(n));
    CHK(ooff.alloc(n + 1));
    CHK(orow_id.alloc(m));
    CHK(osrc.alloc(m));
    const unsigned wgrid = 4096;  // wave-per-row kernels, grid-stride
    if (n) hipLaunchKernelGGL(k_out_count, dim3(wgrid), dim3(TB), 0, s, rp.p, ci.p, n, ocnt.p);
    CHK(exclusive_scan_i32(ocnt.p, ooff.p, n, ooff.p + n, scan_tmp.p, s));
    if (n)
        hipLaunchKernelGGL(k_out_fill, dim3(wgrid), dim3(TB), 0, s, rp.p, ci.p, eid.p, (const int2*)nullptr, n,
                           ooff.p, orow_id.p, osrc.p, 0);
    CHK(hipGetLastError());

    // ---- supports and triangle incidence
    DBuf<int32_t> sup;
    DBuf<int64_t> inc_off, cursor;
    CHK(sup.alloc(m));
    CHK(inc_off.alloc(m + 1));
    CHK(hipMemsetAsync(sup.p, 0, sizeof(int32_t) * (size_t)(m > 0 ? m : 1), s));
    if (m)
        hipLaunchKernelGGL(k_triangles, dim3(grid_for(m)), dim3(TB), 0, s, ooff.p, orow_id.p, osrc.p, m, sup.p,
                           (int64_t*)nullptr, (int2*)nullptr, 0);
    CHK(exclusive_scan_i32(sup.p, inc_off.p, m, inc_off.p + m, scan_tmp.p, s));
    int64_t h_ninc = 0;
    CHK(hipMemcpyAsync(&h_ninc, inc_off.p + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHK(hipMemcpyAsync(hstat + 1, dstat + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    g->max_degree = hstat[1];
    DBuf<int2> inc;
    CHK(inc.alloc(h_ninc));
    CHK(cursor.alloc(m + 1));
    CHK(hipMemcpyAsync(cursor.p, inc_off.p, sizeof(int64_t) * (size_t)(m + 1), hipMemcpyDeviceToDevice, s));
    if (m)
        hipLaunchKernelGGL(k_triangles, dim3(grid_for(m)), dim3(TB), 0, s, ooff.p, orow_id.p, osrc.p, m, sup.p,
                           cursor.p, inc.p, 1);
    CHK(hipGetLastError());
    DBuf<int32_t> sup0;
    CHK(sup0.alloc(m));
    CHK(hipMemcpyAsync(sup0.p, sup.p, sizeof(int32_t) * (size_t)(m > 0 ? m : 1), hipMemcpyDeviceToDevice, s));

    // ---- level-synchronous peel
    DBuf<int32_t> live, keep, front, flag, rnd, level, rank;
    DBuf<int64_t> pos;
    DBuf<PeelState> st;
    CHK(live.alloc(m));
    CHK(keep.alloc(m));
    CHK(front.alloc(m));
    CHK(flag.alloc(m));
    CHK(rnd.alloc(m));
    CHK(level.alloc(m));
    CHK(rank.alloc(m));
    CHK(pos.alloc(m + 1));
    CHK(st.alloc(1));
    PeelState* hst = nullptr;
    CHK(hipHostMalloc((void**)&hst, sizeof(PeelState), hipHostMallocDefault));
    struct HostFree2 { PeelState* p; ~HostFree2() { if (p) (void)hipHostFree(p); } } hf2{hst};
    if (m) {
        hipLaunchKernelGGL(k_iota, dim3(grid_for(m)), dim3(TB), 0, s, live.p, m);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(m)), dim3(TB), 0, s, rnd.p, m, -1);
    }
    int64_t nlive = m, ranked = 0;
    int32_t lev = 0, r = 0, maxlev = 0;
    while (ranked < m) {
        unsigned gl = grid_for(nlive, TB * 8);  // about eight entries per thread
        if (gl > 2048) gl = 2048;
        hipLaunchKernelGGL(k_peel_reset, dim3(1), dim3(1), 0, s, st.p);
        hipLaunchKernelGGL(k_peel_flag, dim3(gl), dim3(TB), 0, s, live.p, nlive, sup.p, lev, flag.p, st.p);
        CHK(exclusive_scan_i32(flag.p, pos.p, nlive, &st.p->nf, scan_tmp.p, s));
        CHK(hipMemcpyAsync(hst, st.p, sizeof(PeelState), hipMemcpyDeviceToHost, s));
        CHK(hipStreamSynchronize(s));
        int64_t nf = hst->nf;
        if (nf == 0) {
            lev = hst->minsup;  // next level that has an edge
            continue;
        }
        hipLaunchKernelGGL(k_peel_compact, dim3(gl), dim3(TB), 0, s, live.p, nlive, flag.p, pos.p, front.p, keep.p);
        unsigned gf = grid_for(nf);
        if (gf > 8192) gf = 8192;
        hipLaunchKernelGGL(k_peel_assign, dim3(gf), dim3(TB), 0, s, front.p, nf, lev, ranked, r, level.p, rank.p,
                           rnd.p);
        unsigned gw = grid_for(nf * EBB_WAVE);
        if (gw > 16384) gw = 16384;
        hipLaunchKernelGGL(k_peel_triangles, dim3(gw), dim3(TB), 0, s, front.p, nf, inc_off.p, inc.p, rnd.p, r,
                           sup.p);
        CHK(hipGetLastError());
        if (lev > maxlev) maxlev = lev;
        ranked += nf;
        nlive -= nf;
        ++r;
        int32_t* t = live.p; live.p = keep.p; keep.p = t;
    }
    g->tau = maxlev;
    g->rounds = r;

    // ---- root edge order from a vertex order (ablation orderings): edges in the
    // lexicographic order of their endpoints' positions replace pi_tau; levels
    // and tau stay those of the truss peel (tau + 2 still bounds the clique size)
    if ((g->opt.ordering == EBBKC_ORDER_COLOR || g->opt.ordering == EBBKC_ORDER_DEGEN_VERTEX ||
         g->opt.ordering == EBBKC_ORDER_DEGEN_VERTEX_NP) && n > 0) {
        const int64_t big = (int64_t)n > m ? (int64_t)n : m;
        DBuf<int32_t> vpos, vcol;
        DBuf<uint64_t> k1, k2;
        DBuf<uint32_t> v1, v2;
        DBuf<int64_t> rh, rht;
        CHK(vpos.alloc(n));
        CHK(k1.alloc(big));
        CHK(k2.alloc(big));
        CHK(v1.alloc(big));
        CHK(v2.alloc(big));
        const int64_t rhn = radix_hist_elems(big);
        CHK(rh.alloc(rhn));
        CHK(rht.alloc(scan_tmp_elems(rhn) + 16));
        if (g->opt.ordering == EBBKC_ORDER_COLOR) {
            // greedy colouring (Section 4.3), then vertices by colour desc, id asc
            CHK(vcol.alloc(n));
            CHK(hipMemsetAsync(vcol.p, 0, sizeof(int32_t) * (size_t)n, s));
            unsigned gc = grid_for((int64_t)n * EBB_WAVE);
            if (gc > 16384) gc = 16384;
            for (;;) {
                CHK(hipMemsetAsync(dstat + 2, 0, sizeof(int), s));
                hipLaunchKernelGGL(k_colour_round, dim3(gc), dim3(TB), 0, s, rp.p, ci.p, n, vcol.p, dstat + 2);
                CHK(hipGetLastError());
                CHK(hipMemcpyAsync(hstat + 2, dstat + 2, sizeof(int), hipMemcpyDeviceToHost, s));
                CHK(hipStreamSynchronize(s));
                if (hstat[2] == 0) break;
            }
            hipLaunchKernelGGL(k_colour_keys, dim3(grid_for(n)), dim3(TB), 0, s, vcol.p, n, k1.p, v1.p);
            CHK(radix_sort_u64(k1.p, v1.p, k2.p, v2.p, n, 31, rh.p, rht.p, s));
            hipLaunchKernelGGL(k_scatter_pos, dim3(grid_for(n)), dim3(TB), 0, s, v1.p, (int64_t)n, vpos.p);
            CHK(hipGetLastError());
        } else {
            // degeneracy order, level-synchronous: at level s every remaining
            // vertex of degree <= s leaves in one round, placed by (round, id)
            DBuf<int32_t> deg, vlive, vkeep, vfront, vflag, vrnd;
            DBuf<int64_t> vps;
            CHK(deg.alloc(n));
            CHK(vlive.alloc(n));
            CHK(vkeep.alloc(n));
            CHK(vfront.alloc(n));
            CHK(vflag.alloc(n));
            CHK(vrnd.alloc(n));
            CHK(vps.alloc(n + 1));
            hipLaunchKernelGGL(k_degrees, dim3(grid_for(n)), dim3(TB), 0, s, rp.p, n, deg.p);
            hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(TB), 0, s, vlive.p, (int64_t)n);
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(TB), 0, s, vrnd.p, (int64_t)n, -1);
            CHK(hipGetLastError());
            int64_t nl = n, placed = 0;
            int32_t lv = 0, rr = 0;
            while (placed < n) {
                unsigned gl = grid_for(nl, TB * 8);
                if (gl > 2048) gl = 2048;
                hipLaunchKernelGGL(k_peel_reset, dim3(1), dim3(1), 0, s, st.p);
                hipLaunchKernelGGL(k_peel_flag, dim3(gl), dim3(TB), 0, s, vlive.p, nl, deg.p, lv, vflag.p, st.p);
                CHK(exclusive_scan_i32(vflag.p, vps.p, nl, &st.p->nf, scan_tmp.p, s));
                CHK(hipMemcpyAsync(hst, st.p, sizeof(PeelState), hipMemcpyDeviceToHost, s));
                CHK(hipStreamSynchronize(s));
                const int64_t nf = hst->nf;
                if (nf == 0) {
                    lv = hst->minsup;
                    continue;
                }
                hipLaunchKernelGGL(k_peel_compact, dim3(gl), dim3(TB), 0, s, vlive.p, nl, vflag.p, vps.p, vfront.p,
                                   vkeep.p);
                hipLaunchKernelGGL(k_core_assign, dim3(grid_for(nf)), dim3(TB), 0, s, vfront.p, nf, placed, rr,
                                   vpos.p, vrnd.p);
                unsigned gw = grid_for(nf * EBB_WAVE);
                if (gw > 16384) gw = 16384;
                hipLaunchKernelGGL(k_core_remove, dim3(gw), dim3(TB), 0, s, vfront.p, nf, rp.p, ci.p, vrnd.p, deg.p);
                CHK(hipGetLastError());
                placed += nf;
                nl -= nf;
                ++rr;
                int32_t* t = vlive.p; vlive.p = vkeep.p; vkeep.p = t;
            }
        }
        if (m) {
            hipLaunchKernelGGL(k_lex_edge_keys, dim3(grid_for(m)), dim3(TB), 0, s, eu.p, ev.p, vpos.p, m, n, k1.p,
                               v1.p);
            CHK(radix_sort_u64(k1.p, v1.p, k2.p, v2.p, m, bits_for((uint64_t)n * (uint64_t)n), rh.p, rht.p, s));
            hipLaunchKernelGGL(k_scatter_pos, dim3(grid_for(m)), dim3(TB), 0, s, v1.p, m, rank.p);
            CHK(hipGetLastError());
        }
        g->vpos = vpos.release();
        g->vcol = vcol.release();
    }

    // ---- rank-tagged adjacency
    DBuf<int32_t> erank;
    DBuf<uint64_t> keys, keys2;
    DBuf<uint32_t> vals, vals2;
    DBuf<int64_t> hist;
    DBuf<int2> rrow, orow;
    DBuf<int32_t> orp, byrank;
    CHK(erank.alloc(nnz));
    CHK(keys.alloc(nnz));
    CHK(keys2.alloc(nnz));
    CHK(vals.alloc(nnz));
    CHK(vals2.alloc(nnz));
    int64_t hn = radix_hist_elems(nnz);
    CHK(hist.alloc(hn));
    DBuf<int64_t> hist_tmp;
    CHK(hist_tmp.alloc(scan_tmp_elems(hn) + 16));
    CHK(rrow.alloc(nnz));
    if (nnz) {
        hipLaunchKernelGGL(k_erank_keys, dim3(grid_for(nnz)), dim3(TB), 0, s, src.p, eid.p, rank.p, nnz, m, erank.p,
                           keys.p, vals.p);
        int bits = bits_for((uint64_t)n * (uint64_t)m);
        CHK(radix_sort_u64(keys.p, vals.p, keys2.p, vals2.p, nnz, bits, hist.p, hist_tmp.p, s));
        hipLaunchKernelGGL(k_gather_rrow, dim3(grid_for(nnz)), dim3(TB), 0, s, vals.p, ci.p, erank.p, nnz, rrow.p);
    }
    CHK(orp.alloc(n + 1));
    CHK(orow.alloc(m));
    if (n) {
        hipLaunchKernelGGL(k_copy_i64_to_i32, dim3(grid_for(n + 1)), dim3(TB), 0, s, ooff.p, orp.p, (int64_t)n + 1);
        hipLaunchKernelGGL(k_out_fill, dim3(wgrid), dim3(TB), 0, s, rp.p, ci.p, eid.p, rrow.p, n, ooff.p, orow.p,
                           (int32_t*)nullptr, 1);
    }
    CHK(byrank.alloc(m));
    if (m) {
        hipLaunchKernelGGL(k_byrank, dim3(grid_for(m)), dim3(TB), 0, s, rank.p, m, byrank.p);
    }
    // ---- adjacency bitmap for sub-branch builds by pair tests (small graphs)
    DBuf<uint64_t> adj;
    DBuf<uint16_t> acum;
    const int32_t amax = g->opt.adj_max_n == 0 ? ADJ_DEFAULT_MAX_N : g->opt.adj_max_n;
    const int32_t aw = (n + 63) / 64;
    const bool with_adj = amax > 0 && n > 0 && n <= amax && m > 0;
    if (with_adj) {
        CHK(adj.alloc((int64_t)n * aw));
        CHK(acum.alloc((int64_t)n * aw));
        CHK(hipMemsetAsync(adj.p, 0, sizeof(uint64_t) * (size_t)n * aw, s));
        hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(nnz)), dim3(TB), 0, s, src.p, ci.p, nnz, aw, adj.p);
        hipLaunchKernelGGL(k_adj_cum, dim3(grid_for((int64_t)n * aw)), dim3(TB), 0, s, rp.p, ci.p, n, aw, acum.p);
    }
    CHK(hipGetLastError());
    CHK(hipEventRecord(ev1, s));
    CHK(hipStreamSynchronize(s));
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    g->prepare_ms = ms;

    g->rp = rp.release();
    g->ci = ci.release();
    g->erank = erank.release();
    g->eu = eu.release();
    g->ev = ev.release();
    g->sup0 = sup0.release();
    g->rank = rank.release();
    g->level = level.release();
    g->rrow = rrow.release();
    g->orp = orp.release();
    g->orow = orow.release();
    g->byrank = byrank.release();
    if (with_adj) {
        g->adj = adj.release();
        g->acum = acum.release();
        g->adjw = aw;
    }
    g->device_bytes = (int64_t)sizeof(int32_t) * ((n + 1) * 2 + nnz * 2 + m * 6) + (int64_t)sizeof(int2) * (nnz + m) +
                      (int64_t)sizeof(int32_t) * n * ((g->vpos ? 1 : 0) + (g->vcol ? 1 : 0)) +
                      (with_adj ? (int64_t)n * aw * (int64_t)(sizeof(uint64_t) + sizeof(uint16_t)) : 0);
    return EBBKC_OK;
}

}  // namespace ebb
