// build.h -- construction of one sub-branch g_i in LDS by one wavefront,
// shared by the arena builder (which then writes g_i to HBM) and the search
// kernel variant that builds each task's g_i in place (batches too large for
// an arena).
//
// For a seed e_i = (u,v) of rank r (Eq. edge-oriented-branching):
//   1. candidates  V(g_i) = {w : (u,w) and (v,w) both ranked after e_i}.  The
//                  shorter of the two rank-sorted row prefixes (entries ranked
//                  after r) is scanned; each entry is looked up in the other
//                  endpoint's id-sorted row, whose rank must also exceed r.
//   2. sub-graph   E(g_i): pairs of V(g_i) joined by an edge ranked after r.
//                  With an adjacency bitmap of G (small graphs), every pair
//                  of members is tested directly (one bit, and for an edge
//                  its rank found from the bitmap's cumulative counts): about
//                  c^2 / 2 tests, against about c times the out-degree for a
//                  scan.  Otherwise every member's degree-oriented row prefix
//                  ranked after r is scanned (all members' prefixes flattened
//                  over the wave's lanes) against an LDS hash of V(g_i); each
//                  such edge is met exactly once.  Both give the same rows.
//   3. colouring   greedy colouring (colours 1, 2, ...) visiting vertices by
//                  non-increasing degree in g_i, ties to the smaller vertex
//                  id (Section 4.3; Algorithm EBBkC-H colours each g_i).
//                  Under EBBkC-C the colours of G's own colouring are kept
//                  instead (renumbered 1..D among the colours present).
//   4. order       position of every vertex when sorted by non-increasing
//                  colour, ties to the smaller vertex id (the DAG of
//                  Algorithm EBBkC-H orients edges low -> high in it).
#pragma once
#include "arena.h"
#include "device_util.h"

namespace ebb {

template <int W>
constexpr int hash_size() { return W <= 1 ? 128 : (W <= 2 ? 256 : 512); }

// LDS bytes of the build's work areas (BuildScratch) for width class W
template <int W>
constexpr int build_scratch_bytes() { return 4 * 64 * W + 4 * 64 * W + 4 * hash_size<W>() + 2 * hash_size<W>() + 2 * 64 * W; }

__device__ __forceinline__ uint32_t hslot(int32_t key, int hs) {
    return ((uint32_t)key * 2654435761u) & (uint32_t)(hs - 1);
}

// The build's LDS work areas: candidate ids, a per-vertex key, the open
// addressing hash (id -> local index) and a visiting sequence.
template <int W>
struct BuildScratch {
    int32_t* gid;   // [64 W]
    int32_t* key;   // [64 W]
    int32_t* hkey;  // [hash_size]
    int16_t* hval;  // [hash_size]
    int16_t* seq;   // [64 W]
    // carve the areas out of `base` (4-byte aligned, build_scratch_bytes<W>() bytes)
    __device__ static BuildScratch carve(void* base) {
        char* p = reinterpret_cast<char*>(base);
        BuildScratch S;
        S.gid = reinterpret_cast<int32_t*>(p);
        p += 4 * 64 * W;
        S.key = reinterpret_cast<int32_t*>(p);
        p += 4 * 64 * W;
        S.hkey = reinterpret_cast<int32_t*>(p);
        p += 4 * hash_size<W>();
        S.hval = reinterpret_cast<int16_t*>(p);
        p += 2 * hash_size<W>();
        S.seq = reinterpret_cast<int16_t*>(p);
        return S;
    }
};

template <int W>
__device__ __forceinline__ int hash_find(const BuildScratch<W>& S, int32_t key) {
    constexpr int HS = hash_size<W>();
    uint32_t h = hslot(key, HS);
    for (int t = 0; t < HS; ++t) {
        int32_t kk = S.hkey[h];
        if (kk == key) return S.hval[h];
        if (kk < 0) return -1;
        h = (h + 1) & (HS - 1);
    }
    return -1;
}

// Whether (x, w) is an edge of G ranked after r: a bit of the adjacency
// bitmap, then the edge's rank at its position in the id-sorted row (the
// entries before its word plus the set bits below it in the word); without
// a bitmap, by binary search of the id-sorted row.
__device__ __forceinline__ bool later_edge(const GraphView& G, int32_t x, int32_t w, int32_t r) {
    if (G.adj) {
        const int64_t o = (int64_t)x * G.adjw + (w >> 6);
        const uint64_t word = G.adj[o];
        if (!((word >> (w & 63)) & 1)) return false;
        return G.erank[G.rp[x] + (int)G.acum[o] + popc64(word & ((1ull << (w & 63)) - 1))] > r;
    }
    const int q = lower_bound_i32(G.ci, G.rp[x], G.rp[x + 1], w);
    return q < G.rp[x + 1] && G.ci[q] == w && G.erank[q] > r;
}

// later_edge for PB pairs (x[t], w[t]) at once: with the bitmap, every load
// of the first step (bitmap word, row start, entries before the word) is
// issued before any is used, then the rank loads of the pairs that are edges,
// so the PB chains of dependent loads overlap instead of following each other.
template <int PB>
__device__ __forceinline__ void later_edges(const GraphView& G, const int32_t (&x)[PB], const int32_t (&w)[PB],
                                            const bool (&valid)[PB], int32_t r, bool (&ok)[PB]) {
    if (G.adj) {
        uint64_t word[PB];
        int32_t row0[PB], below[PB];
#pragma unroll
        for (int t = 0; t < PB; ++t) {
            word[t] = 0;
            row0[t] = 0;
            below[t] = 0;
            if (valid[t]) {
                const int64_t o = (int64_t)x[t] * G.adjw + (w[t] >> 6);
                word[t] = G.adj[o];
                row0[t] = G.rp[x[t]];
                below[t] = (int32_t)G.acum[o];
            }
        }
#pragma unroll
        for (int t = 0; t < PB; ++t) {
            ok[t] = false;
            if (valid[t] && ((word[t] >> (w[t] & 63)) & 1))
                ok[t] = G.erank[row0[t] + below[t] + popc64(word[t] & ((1ull << (w[t] & 63)) - 1))] > r;
        }
    } else {
#pragma unroll
        for (int t = 0; t < PB; ++t) ok[t] = valid[t] && later_edge(G, x[t], w[t], r);
    }
}

// pairs (or row entries) a lane tests per round of the build
constexpr int BUILD_PB = 4;

// number of entries of row x (rank-sorted, descending) ranked after r
__device__ __forceinline__ int prefix_after(const int32_t* __restrict__ rp, const int2* __restrict__ rrow, int32_t x,
                                            int32_t r) {
    int lo = rp[x], hi = rp[x + 1];
    const int base = lo;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (rrow[mid].y > r) lo = mid + 1; else hi = mid;
    }
    return lo - base;
}

// Steps 1-3 for the seed (u, v) of rank r (a vertex slot passes u = v and the
// rank threshold of its out-edges): candidates into S.gid, their symmetric
// adjacency bitmap into rows (candidate order), colours into col.  Returns
// c = |V(g_i)| (uniform), or -1 when c exceeds 64 W or differs from expect
// (expect < 0: not checked); *twoE = 2 |E(g_i)|.
template <int W>
__device__ int build_subbranch(const GraphView& G, int32_t u, int32_t v, int32_t r, int expect,
                               const int32_t* __restrict__ vcol, uint64_t (*rows)[W], int16_t* col,
                               const BuildScratch<W>& S, uint32_t* twoE) {
    const int lane = lane_id();
    constexpr int CAP = 64 * W;
    constexpr int HS = hash_size<W>();

    // ---- 1. candidates
    const int lu = prefix_after(G.rp, G.rrow, u, r), lv = prefix_after(G.rp, G.rrow, v, r);
    const int32_t xs = lu <= lv ? u : v, ys = lu <= lv ? v : u;
    const int lx = lu <= lv ? lu : lv;
    int c = 0;
    const int32_t xrow = G.rp[xs];
    for (int base = 0; base < lx; base += 64 * BUILD_PB) {
        int32_t wv[BUILD_PB], yv[BUILD_PB];
        bool val[BUILD_PB], okv[BUILD_PB];
#pragma unroll
        for (int t = 0; t < BUILD_PB; ++t) {
            const int idx = base + 64 * t + lane;
            val[t] = idx < lx;
            wv[t] = val[t] ? G.rrow[xrow + idx].x : -1;
            yv[t] = ys;
        }
        later_edges<BUILD_PB>(G, yv, wv, val, r, okv);
#pragma unroll
        for (int t = 0; t < BUILD_PB; ++t) {  // in row order, as one entry per lane per round
            const uint64_t mk = ballot(okv[t]);
            if (okv[t]) {
                const int p = c + popc64(mk & lanemask_lt());
                if (p < CAP) S.gid[p] = wv[t];
            }
            c += popc64(mk);
        }
    }
    c = uniform_i32(c);
    if (c > CAP || (expect >= 0 && c != expect)) return -1;

    // ---- 2. sub-graph bitmap
    for (int i = lane; i < c; i += 64)
#pragma unroll
        for (int w = 0; w < W; ++w) rows[i][w] = 0;
    if (G.adj) {
        wave_sync();
        const int U = c * (c - 1) / 2;
        for (int u0 = 0; u0 < U; u0 += 64 * BUILD_PB) {
            int pi[BUILD_PB], pj[BUILD_PB];
            int32_t xa[BUILD_PB], wb[BUILD_PB];
            bool val[BUILD_PB], okv[BUILD_PB];
#pragma unroll
            for (int t = 0; t < BUILD_PB; ++t) {
                const int u = u0 + 64 * t + lane;
                val[t] = u < U;
                pi[t] = 0;
                pj[t] = 0;
                if (val[t]) upper_pair(u, c, pi[t], pj[t]);
                xa[t] = val[t] ? S.gid[pi[t]] : 0;
                wb[t] = val[t] ? S.gid[pj[t]] : 0;
            }
            later_edges<BUILD_PB>(G, xa, wb, val, r, okv);
#pragma unroll
            for (int t = 0; t < BUILD_PB; ++t) {
                if (okv[t]) {
                    atomicOr((unsigned long long*)&rows[pi[t]][pj[t] >> 6], 1ull << (pj[t] & 63));
                    atomicOr((unsigned long long*)&rows[pj[t]][pi[t] >> 6], 1ull << (pi[t] & 63));
                }
            }
        }
    } else {
        for (int j = lane; j < HS; j += 64) S.hkey[j] = -1;
        wave_sync();
        for (int i = lane; i < c; i += 64) {
            const int32_t key = S.gid[i];
            uint32_t h = hslot(key, HS);
            while (true) {
                const int32_t old = atomicCAS(&S.hkey[h], -1, key);
                if (old == -1) { S.hval[h] = (int16_t)i; break; }
                h = (h + 1) & (HS - 1);
            }
        }
        wave_sync();
        {
            int plen[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int i = lane + 64 * q;
                plen[q] = 0;
                if (i < c) {
                    const int32_t w = S.gid[i];
                    int lo = G.orp[w], hi = G.orp[w + 1];
                    const int base = lo;
                    while (lo < hi) {
                        int mid = (lo + hi) >> 1;
                        if (G.orow[mid].y > r) lo = mid + 1; else hi = mid;
                    }
                    plen[q] = lo - base;
                }
            }
            int total = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int inc = wave_incl_scan(plen[q]);
                const int i = lane + 64 * q;
                if (i < c) S.key[i] = total + inc - plen[q];
                total += __shfl(inc, 63, 64);
            }
            wave_sync();
            for (int base = 0; base < total; base += 64) {
                const int j = base + lane;
                if (j < total) {
                    int lo = 0, hi = c;  // last member whose offset is <= j
                    while (hi - lo > 1) {
                        int mid = (lo + hi) >> 1;
                        if (S.key[mid] <= j) lo = mid; else hi = mid;
                    }
                    const int i = lo;
                    const int2 yr = G.orow[G.orp[S.gid[i]] + (j - S.key[i])];
                    const int jj = hash_find(S, yr.x);
                    if (jj >= 0) {
                        atomicOr((unsigned long long*)&rows[i][jj >> 6], 1ull << (jj & 63));
                        atomicOr((unsigned long long*)&rows[jj][i >> 6], 1ull << (i & 63));
                    }
                }
            }
        }
    }
    wave_sync();

    // ---- 3a. colouring order: degree desc, id asc
    uint32_t dsum = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const int i = lane + 64 * q;
        if (i < c) {
            int d = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) d += popc64(rows[i][w]);
            S.key[i] = d;
            dsum += d;
        }
    }
    *twoE = wave_sum(dsum);
    wave_sync();
    if (vcol) {
        // ---- 3'. G's colouring kept (EBBkC-C): the colours present are
        // renumbered 1..D in their order, which changes neither the order
        // below nor the number of colours in any vertex set
        for (int i = lane; i < c; i += 64) S.key[i] = vcol[S.gid[i]];
        wave_sync();
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int i = lane + 64 * q;
            const int ki = i < c ? S.key[i] : 0, gi = i < c ? S.gid[i] : 0;
            int ord = 0;
            for (int j = 0; j < c; ++j) {
                const int kj = S.key[j], gj = S.gid[j];
                ord += (kj > ki) || (kj == ki && gj < gi);
            }
            if (i < c) S.seq[ord] = (int16_t)i;
        }
        wave_sync();
        int cum[W];
        int starts = 0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int p = lane + 64 * q;
            const bool st = p < c && (p == 0 || S.key[S.seq[p]] != S.key[S.seq[p - 1]]);
            const uint64_t mk = ballot(st);
            cum[q] = starts + popc64(mk & (lanemask_lt() | (1ull << lane)));
            starts += popc64(mk);
        }
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int p = lane + 64 * q;
            if (p < c) col[S.seq[p]] = (int16_t)(starts - cum[q] + 1);
        }
        wave_sync();
    } else {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int i = lane + 64 * q;
            const int di = i < c ? S.key[i] : 0, gi = i < c ? S.gid[i] : 0;
            int ord = 0;
            for (int j = 0; j < c; ++j) {
                const int dj = S.key[j], gj = S.gid[j];
                ord += (dj > di) || (dj == di && gj < gi);
            }
            if (i < c) S.seq[ord] = (int16_t)i;
        }
        wave_sync();
        // ---- 3b. greedy colouring; colour-class masks live in lanes
        uint64_t cls[W][W];
#pragma unroll
        for (int q = 0; q < W; ++q)
#pragma unroll
            for (int w = 0; w < W; ++w) cls[q][w] = 0;
        int ncol = 0;
        for (int t = 0; t < c; ++t) {
            const int i = S.seq[t];
            uint64_t A[W];
#pragma unroll
            for (int w = 0; w < W; ++w) A[w] = rows[i][w];
            int found = -1;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                bool ok = lane + 64 * q < ncol;
#pragma unroll
                for (int w = 0; w < W; ++w) ok = ok && ((cls[q][w] & A[w]) == 0);
                const uint64_t mk = ballot(ok);
                if (found < 0 && mk) found = 64 * q + __builtin_ctzll(mk);
            }
            if (found < 0) found = ncol++;
            found = uniform_i32(found);
            if (lane == (found & 63)) {
#pragma unroll
                for (int q = 0; q < W; ++q)
                    if (q == (found >> 6)) {
#pragma unroll
                        for (int w = 0; w < W; ++w)
                            if (w == (i >> 6)) cls[q][w] |= 1ull << (i & 63);
                    }
            }
            if (lane == 0) col[i] = (int16_t)(found + 1);
        }
        wave_sync();
    }
    return c;
}

// Step 4: npos[q] = position of local vertex lane + 64 q in the order by
// non-increasing colour, ties to the smaller global id (also stored in S.key).
template <int W>
__device__ __forceinline__ void order_positions(int c, const int16_t* col, const BuildScratch<W>& S, int (&npos)[W]) {
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const int i = lane + 64 * q;
        const int ci_ = i < c ? col[i] : 0, gi = i < c ? S.gid[i] : 0;
        int ord = 0;
        for (int j = 0; j < c; ++j) {
            const int cj = col[j], gj = S.gid[j];
            ord += (cj > ci_) || (cj == ci_ && gj < gi);
        }
        npos[q] = ord;
        if (i < c) S.key[i] = ord;
    }
    wave_sync();
}

// Row of local vertex i with its bits moved to the vertices' positions
template <int W>
__device__ __forceinline__ void relabelled_row(const uint64_t (*rows)[W], int i, const BuildScratch<W>& S,
                                               uint64_t (&nr)[W]) {
#pragma unroll
    for (int w = 0; w < W; ++w) nr[w] = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t b = rows[i][w];
        while (b) {
            const int j = w * 64 + __builtin_ctzll(b);
            b &= b - 1;
            const int pj = S.key[j];
#pragma unroll
            for (int ww = 0; ww < W; ++ww)
                if (ww == (pj >> 6)) nr[ww] |= 1ull << (pj & 63);
        }
    }
}

}  // namespace ebb
