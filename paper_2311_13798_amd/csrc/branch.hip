// branch.hip -- the EBBkC-H branch engine: one wavefront per seed edge.
//
// For a seed e_i = (u,v) of rank r (Eq. edge-oriented-branching):
//   1. candidates  C = {w : (u,w) and (v,w) both ranked after e_i}.  The
//                  shorter of the two rank-sorted prefixes (entries ranked
//                  after r) is scanned; each entry is looked up in the other
//                  endpoint's id-sorted row, whose rank must also exceed r.
//   2. sub-graph   g_i: pairs of C joined by an edge ranked after r, found
//                  by scanning each member's degree-oriented row prefix
//                  (ranked after r) against an LDS hash of C; stored as a
//                  symmetric bitmap, 64*W vertices at most.
//   3. colouring   greedy colouring visiting vertices by non-increasing degree
//                  in g_i (ties: smaller vertex id), colours 1,2,...; then the
//                  vertices are relabelled by non-increasing colour (ties:
//                  smaller vertex id) and oriented low -> high (Section 4.3,
//                  Algorithm EBBkC-H).
//   4. search      EBBkC-C_Rec on the DAG: a node (P, l) with |P| < l is
//                  pruned; l = 1 and l = 2 are counted directly (Algorithm
//                  EBBkC); at l >= 3 a clique or 2-plex candidate set is
//                  finished in closed form (Section 5); otherwise every DAG
//                  edge x->y inside P spawns P' = P & N+(x) & N+(y), l-2,
//                  skipped by Rule (1) (col x < l or col y < l-1) and Rule (2)
//                  (fewer than l-2 colours in P').
// The whole wave works on one node at a time: lanes own vertices (rows of
// the bitmap) and the child loop is wave-uniform.
#include "branch.h"
#include "common.h"
#include "handle.h"

namespace ebb {

// C(n, r) for n < BIN_N, r < BIN_R, saturated to UINT64_MAX when it does not fit
constexpr int BIN_N = 1025, BIN_R = 65;
__device__ uint64_t g_binom[BIN_N * BIN_R];

__global__ void k_binom_init() {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= BIN_N) return;
    // row n by the multiplicative recurrence in 128 bits
    unsigned __int128 c = 1;
    bool sat = false;
    g_binom[n * BIN_R + 0] = 1;
    for (int r = 1; r < BIN_R; ++r) {
        if (r > n) { g_binom[n * BIN_R + r] = 0; continue; }
        if (!sat) {
            c = c * (unsigned __int128)(n - r + 1) / (unsigned __int128)r;
            if (c > (unsigned __int128)UINT64_MAX) sat = true;
        }
        g_binom[n * BIN_R + r] = sat ? UINT64_MAX : (uint64_t)c;
    }
}

namespace {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// C(n, r) or UINT64_MAX if it does not fit 64 bits
__device__ uint64_t binom(int n, int r) {
    if (r < 0 || r > n) return 0;
    if (r > n - r) r = n - r;
    if (n < BIN_N && r < BIN_R) return g_binom[n * BIN_R + r];
    unsigned __int128 c = 1;
    for (int j = 1; j <= r; ++j) {
        c = c * (unsigned __int128)(n - r + j) / (unsigned __int128)j;
        if (c > (unsigned __int128)UINT64_MAX) return UINT64_MAX;
    }
    return (uint64_t)c;
}

// a*b with saturation
__device__ __forceinline__ uint64_t mul_sat(uint64_t a, uint64_t b) {
    if (a == 0 || b == 0) return 0;
    if (a == UINT64_MAX || b == UINT64_MAX) return UINT64_MAX;
    uint64_t hi = __umul64hi(a, b);
    return hi ? UINT64_MAX : a * b;
}
__device__ __forceinline__ uint64_t add_sat(uint64_t a, uint64_t b) {
    uint64_t c = a + b;
    return (c < a || a == UINT64_MAX || b == UINT64_MAX) ? UINT64_MAX : c;
}

// l-cliques of a 2-plex with f vertices adjacent to all others and p
// non-adjacent pairs: sum_j C(p,j) 2^j C(f, l-j) (closed form of kC2Plex)
__device__ uint64_t twoplex_count(int f, int p, int l) {
    uint64_t s = 0;
    int jmax = p < l ? p : l;
    for (int j = 0; j <= jmax; ++j) {
        if (l - j > f) continue;
        uint64_t t = mul_sat(binom(p, j), binom(f, l - j));
        t = (j >= 64) ? (t ? UINT64_MAX : 0) : mul_sat(t, 1ull << j);
        s = add_sat(s, t);
    }
    return s;
}

// bits strictly above x within word w of a W-word row
__device__ __forceinline__ uint64_t upper_mask(int x, int w) {
    int xw = x >> 6, xb = x & 63;
    if (w < xw) return 0;
    if (w > xw) return ~0ull;
    return xb == 63 ? 0ull : (~0ull << (xb + 1));
}

template <int W>
struct Frame {
    uint64_t P[W];
    uint64_t R[W];
    int32_t x;
    int32_t l;
    int32_t px, py;  // the DAG edge that produced this node (listing)
};

template <int W>
struct WaveMem {
    uint64_t rows[64 * W][W];
    int32_t gid[64 * W];
    int32_t key[64 * W];
    int32_t hkey[(W <= 1 ? 128 : (W <= 2 ? 256 : 512))];
    int16_t hval[(W <= 1 ? 128 : (W <= 2 ? 256 : 512))];
    int16_t seq[64 * W];
    int16_t col[64 * W];
    Frame<W> fr[MAX_FRAMES];
};

template <int W>
constexpr int hash_size() { return W <= 1 ? 128 : (W <= 2 ? 256 : 512); }

__device__ __forceinline__ uint32_t hslot(int32_t key, int hs) { return ((uint32_t)key * 2654435761u) & (uint32_t)(hs - 1); }

template <int W>
__device__ __forceinline__ int hash_find(const WaveMem<W>& M, int32_t key) {
    constexpr int HS = hash_size<W>();
    uint32_t h = hslot(key, HS);
    for (int t = 0; t < HS; ++t) {
        int32_t kk = M.hkey[h];
        if (kk == key) return M.hval[h];
        if (kk < 0) return -1;
        h = (h + 1) & (HS - 1);
    }
    return -1;
}

// Per-wave search state held in registers: lane-owned rows of the bitmap.
template <int W>
struct Lanes {
    uint64_t srow[W][W];  // symmetric row of vertex lane + 64 q
    uint64_t cls[W][W];   // vertex mask of colour class lane + 64 q (colour lane + 64 q + 1)
};

struct Acc {
    uint64_t lo, hi;
    __device__ void add(uint64_t v) {
        uint64_t o = lo;
        lo += v;
        if (lo < o) ++hi;
        if (v == UINT64_MAX) hi |= 1ull << 62;  // saturated term: overflow marker
    }
};

template <int W>
__device__ __forceinline__ int popcW(const uint64_t (&p)[W]) {
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) c += popc64(p[w]);
    return c;
}

// ----------------------------------------------------------- node kernels

// sum over x in P of |P & N+(x)|  (l = 2)
template <int W>
__device__ __forceinline__ uint64_t edges_in(const Lanes<W>& L, const uint64_t (&P)[W]) {
    int lane = lane_id();
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        int x = lane + 64 * q;
        if ((P[q] >> lane) & 1) {
#pragma unroll
            for (int w = 0; w < W; ++w) c += popc64(P[w] & L.srow[q][w] & upper_mask(x, w));
        }
    }
    return (uint64_t)wave_sum(c);
}

template <int W>
__device__ __forceinline__ void deg_stats(const Lanes<W>& L, const uint64_t (&P)[W], int pc, int& mind, int& nfull) {
    int lane = lane_id();
    int mn = 1 << 30, nf = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        if ((P[q] >> lane) & 1) {
            int d = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) d += popc64(P[w] & L.srow[q][w]);
            mn = d < mn ? d : mn;
            nf += (d == pc - 1);
        }
    }
    mind = wave_min(mn);
    nfull = wave_sum(nf);
}

template <int W>
__device__ __forceinline__ int distinct_colours(const Lanes<W>& L, const uint64_t (&P)[W]) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        uint64_t hit = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) hit |= P[w] & L.cls[q][w];
        c += popc64(ballot(hit != 0));
    }
    return c;
}

}  // namespace

template <int W, bool LIST>
__global__ __launch_bounds__(256) void k_branch(BranchArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    WaveMem<W>& M = reinterpret_cast<WaveMem<W>*>(smem_raw)[threadIdx.x / 64];
    Frame<W>* gfr = a.gframes ? reinterpret_cast<Frame<W>*>(a.gframes) +
                                    ((int64_t)blockIdx.x * 4 + threadIdx.x / 64) * GLOBAL_FRAMES
                              : nullptr;
    // frames beyond the LDS ones live in this wave's slab of device memory;
    // every lane writes them (identical values), so each lane reads its own stores
    auto FR = [&](int d) -> Frame<W>& { return d < MAX_FRAMES ? M.fr[d] : gfr[d - MAX_FRAMES]; };
    const int lane = lane_id();
    constexpr int CAP = 64 * W;
    constexpr int HS = hash_size<W>();
    const int k = a.k;
    const int opts = a.opts;
    const bool rule1 = opts & OPT_RULE1, rule2 = opts & OPT_RULE2, et = opts & OPT_ET, t2 = opts & OPT_TPLEX2;
    const bool work = opts & OPT_WORK;
    Acc acc{0, 0};
    uint64_t wk_seeds = 0, wk_nodes = 0, wk_ops = 0;  // uniform search-work counters

    for (;;) {
        unsigned long long it = 0;
        if (lane == 0) it = atomicAdd(a.next, 1ull);
        it = uni64(__shfl(it, 0, 64));
        if ((int64_t)it >= a.nseeds) break;
        const int64_t si = a.reverse ? a.nseeds - 1 - (int64_t)it : (int64_t)it;
        const int64_t oi = a.out_index ? a.out_index[si] : a.out_base + si;
        const int32_t e = a.seeds[si];
        const int32_t u = a.eu[e], v = a.ev[e], r = a.rank[e];
        Acc sacc{0, 0};

        // ---- 1. candidates: shorter rank-sorted prefix, looked up in the other row
        int lu, lv;
        {
            // prefix length = number of entries with rank > r (ranks descending)
            int lo = a.rp[u], hi = a.rp[u + 1];
            while (lo < hi) { int mid = (lo + hi) >> 1; if (a.rrow[mid].y > r) lo = mid + 1; else hi = mid; }
            lu = lo - a.rp[u];
            lo = a.rp[v]; hi = a.rp[v + 1];
            while (lo < hi) { int mid = (lo + hi) >> 1; if (a.rrow[mid].y > r) lo = mid + 1; else hi = mid; }
            lv = lo - a.rp[v];
        }
        const int32_t xs = lu <= lv ? u : v, ys = lu <= lv ? v : u;
        const int lx = lu <= lv ? lu : lv;
        int c = 0;
        for (int base = 0; base < lx; base += 64) {
            int idx = base + lane;
            bool ok = false;
            int32_t w = -1;
            if (idx < lx) {
                w = a.rrow[a.rp[xs] + idx].x;
                int q = lower_bound_i32(a.ci, a.rp[ys], a.rp[ys + 1], w);
                ok = q < a.rp[ys + 1] && a.ci[q] == w && a.erank[q] > r;
            }
            uint64_t mk = ballot(ok);
            if (ok) {
                int p = c + popc64(mk & lanemask_lt());
                if (p < CAP) M.gid[p] = w;
            }
            c += popc64(mk);
        }
        c = uniform_i32(c);
        if (c > CAP) {
            if (lane == 0) atomicOr(a.err, ERR_WIDTH);
            continue;
        }
        if (c < k - 2) {
            if (!LIST && a.per_seed && lane == 0) a.per_seed[oi] = 0;
            continue;
        }
        wave_sync();
        wk_seeds += work;
        if (k == 3) {
            sacc.add((uint64_t)c);
            goto seed_done;
        }

        // ---- 2. sub-graph bitmap
        for (int j = lane; j < HS; j += 64) M.hkey[j] = -1;
        for (int i = lane; i < c; i += 64)
#pragma unroll
            for (int w = 0; w < W; ++w) M.rows[i][w] = 0;
        wave_sync();
        for (int i = lane; i < c; i += 64) {
            int32_t key = M.gid[i];
            uint32_t h = hslot(key, HS);
            while (true) {
                int32_t old = atomicCAS(&M.hkey[h], -1, key);
                if (old == -1) { M.hval[h] = (int16_t)i; break; }
                h = (h + 1) & (HS - 1);
            }
        }
        wave_sync();
        for (int i = lane; i < c; i += 64) {
            int32_t w = M.gid[i];
            for (int t = a.orp[w]; t < a.orp[w + 1]; ++t) {
                int2 yr = a.orow[t];
                if (yr.y <= r) break;  // rows are sorted by rank, descending
                int j = hash_find(M, yr.x);
                if (j >= 0) {
                    atomicOr((unsigned long long*)&M.rows[i][j >> 6], 1ull << (j & 63));
                    atomicOr((unsigned long long*)&M.rows[j][i >> 6], 1ull << (i & 63));
                }
            }
        }
        wave_sync();

        {
            Lanes<W> L;
            // ---- 3a. colouring order: degree desc, id asc
#pragma unroll
            for (int q = 0; q < W; ++q) {
                int i = lane + 64 * q;
                if (i < c) {
                    int d = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) d += popc64(M.rows[i][w]);
                    M.key[i] = d;
                }
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < W; ++q) {
                int i = lane + 64 * q;
                int di = i < c ? M.key[i] : 0, gi = i < c ? M.gid[i] : 0, ord = 0;
                for (int j = 0; j < c; ++j) {
                    int dj = M.key[j], gj = M.gid[j];
                    ord += (dj > di) || (dj == di && gj < gi);
                }
                if (i < c) M.seq[ord] = (int16_t)i;
            }
            wave_sync();
            // ---- 3b. greedy colouring; class masks live in lanes
#pragma unroll
            for (int q = 0; q < W; ++q)
#pragma unroll
                for (int w = 0; w < W; ++w) L.cls[q][w] = 0;
            int ncol = 0;
            for (int t = 0; t < c; ++t) {
                int i = M.seq[t];
                uint64_t A[W];
#pragma unroll
                for (int w = 0; w < W; ++w) A[w] = M.rows[i][w];
                int found = -1;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    bool ok = lane + 64 * q < ncol;
#pragma unroll
                    for (int w = 0; w < W; ++w) ok = ok && ((L.cls[q][w] & A[w]) == 0);
                    uint64_t mk = ballot(ok);
                    if (found < 0 && mk) found = 64 * q + __builtin_ctzll(mk);
                }
                if (found < 0) found = ncol++;
                found = uniform_i32(found);
                if (lane == (found & 63)) {
#pragma unroll
                    for (int q = 0; q < W; ++q)
                        if (q == (found >> 6)) L.cls[q][i >> 6] |= 1ull << (i & 63);
                }
                if (lane == 0) M.col[i] = (int16_t)(found + 1);
            }
            wave_sync();
            // ---- 3c. relabel by colour desc, id asc
            int npos[W];
            int32_t mygid[W];
            int16_t mycol[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                int i = lane + 64 * q;
                int ci_ = i < c ? M.col[i] : 0, gi = i < c ? M.gid[i] : 0, ord = 0;
                for (int j = 0; j < c; ++j) {
                    int cj = M.col[j], gj = M.gid[j];
                    ord += (cj > ci_) || (cj == ci_ && gj < gi);
                }
                npos[q] = ord;
                mygid[q] = gi;
                mycol[q] = (int16_t)ci_;
                if (i < c) M.key[i] = ord;
            }
            wave_sync();
            uint64_t nr[W][W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                int i = lane + 64 * q;
#pragma unroll
                for (int w = 0; w < W; ++w) nr[q][w] = 0;
                if (i < c) {
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        uint64_t b = M.rows[i][w];
                        while (b) {
                            int j = w * 64 + __builtin_ctzll(b);
                            b &= b - 1;
                            int pj = M.key[j];
#pragma unroll
                            for (int ww = 0; ww < W; ++ww)
                                if (ww == (pj >> 6)) nr[q][ww] |= 1ull << (pj & 63);
                        }
                    }
                }
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < W; ++q) {
                int i = lane + 64 * q;
                if (i < c) {
#pragma unroll
                    for (int w = 0; w < W; ++w) M.rows[npos[q]][w] = nr[q][w];
                    M.gid[npos[q]] = mygid[q];
                    M.col[npos[q]] = mycol[q];
                }
            }
            wave_sync();
            // lane-owned symmetric rows and colour-class masks (relabelled)
#pragma unroll
            for (int q = 0; q < W; ++q) {
                int x = lane + 64 * q;
#pragma unroll
                for (int w = 0; w < W; ++w) L.srow[q][w] = x < c ? M.rows[x][w] : 0;
            }
            // class of colour cv occupies relabelled positions [#(col > cv), #(col >= cv))
#pragma unroll
            for (int q = 0; q < W; ++q) {
                int cv = lane + 64 * q + 1;
                int lo = 0, hi = c;  // first position with col <= cv (col non-increasing)
                while (lo < hi) { int mid = (lo + hi) >> 1; if (M.col[mid] > cv) lo = mid + 1; else hi = mid; }
                int s0 = lo;
                lo = s0; hi = c;
                while (lo < hi) { int mid = (lo + hi) >> 1; if (M.col[mid] >= cv) lo = mid + 1; else hi = mid; }
                int s1 = cv <= ncol ? lo : s0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    int a0 = s0 > 64 * w ? s0 : 64 * w, a1 = s1 < 64 * w + 64 ? s1 : 64 * w + 64;
                    uint64_t mk = 0;
                    if (a1 > a0) {
                        int len = a1 - a0;
                        mk = (len == 64 ? ~0ull : ((1ull << len) - 1)) << (a0 - 64 * w);
                    }
                    L.cls[q][w] = mk;
                }
            }

            // ---- 4. search
            const int l0 = k - 2;
            uint64_t P0[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                int lo = 64 * w;
                P0[w] = c >= lo + 64 ? ~0ull : (c > lo ? ((1ull << (c - lo)) - 1) : 0ull);
            }
            int sp = 0;
            // evaluate one node: count it, or push a frame to expand it
            auto node = [&](const uint64_t (&P)[W], int l, int px, int py) {
                int pc = popcW(P);
                if (work) { wk_nodes += 1; wk_ops += W; }
                if (pc < l) return;
                if (l == 1) {
                    sacc.add((uint64_t)pc);
                    return;
                }
                if (l == 2) {
                    if (work) wk_ops += (uint64_t)pc * W;
                    sacc.add(edges_in(L, P));
                    return;
                }
                if (et) {
                    if (work) wk_ops += (uint64_t)pc * W;
                    int mind, nfull;
                    deg_stats(L, P, pc, mind, nfull);
                    if (mind >= pc - 1) { sacc.add(binom(pc, l)); return; }
                    if (t2 && mind >= pc - 2) { sacc.add(twoplex_count(nfull, (pc - nfull) / 2, l)); return; }
                }
                if (l == 3) {
                    // triangles of the DAG inside P: lanes own x, y runs over P
                    uint64_t R[W][W];
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        int x = lane + 64 * q;
                        bool in = ((P[q] >> lane) & 1) && !(rule1 && x < c && M.col[x] < 3);
#pragma unroll
                        for (int w = 0; w < W; ++w) R[q][w] = in ? (P[w] & L.srow[q][w] & upper_mask(x, w)) : 0;
                    }
                    uint32_t cnt = 0;
                    bool stop = false;
#pragma unroll
                    for (int wy = 0; wy < W; ++wy) {
                        uint64_t bits = stop ? 0ull : P[wy];
                        while (bits) {
                            int y = wy * 64 + __builtin_ctzll(bits);
                            bits &= bits - 1;
                            if (rule1 && M.col[y] < 2) { stop = true; break; }
                            uint64_t Uy[W];
#pragma unroll
                            for (int w = 0; w < W; ++w) Uy[w] = M.rows[y][w] & upper_mask(y, w);
#pragma unroll
                            for (int q = 0; q < W; ++q) {
                                bool act = (R[q][y >> 6] >> (y & 63)) & 1;
                                if (work) wk_ops += (uint64_t)popc64(ballot(act)) * W;
                                if (act) {
#pragma unroll
                                    for (int w = 0; w < W; ++w) cnt += popc64(R[q][w] & Uy[w]);
                                }
                            }
                        }
                    }
                    sacc.add((uint64_t)wave_sum(cnt));
                    return;
                }
                if (sp >= MAX_FRAMES + (gfr ? GLOBAL_FRAMES : 0)) {
                    if (lane == 0) atomicOr(a.err, ERR_DEPTH);
                    return;
                }
                if (lane == 0 || sp >= MAX_FRAMES) {
                    Frame<W>& F = FR(sp);
#pragma unroll
                    for (int w = 0; w < W; ++w) { F.P[w] = P[w]; F.R[w] = 0; }
                    F.x = -1;
                    F.l = l;
                    F.px = px;
                    F.py = py;
                }
                ++sp;
                wave_sync();
            };

            node(P0, l0, -1, -1);
            while (sp > 0) {
                Frame<W>& F = FR(sp - 1);
                uint64_t P[W], R[W];
#pragma unroll
                for (int w = 0; w < W; ++w) { P[w] = uni64(F.P[w]); R[w] = uni64(F.R[w]); }
                int x = uniform_i32(F.x), l = uniform_i32(F.l);
                int y = -1;
                bool done = false;
                while (true) {
                    bool any = false;
#pragma unroll
                    for (int w = 0; w < W; ++w) any |= R[w] != 0;
                    if (any) {
                        int wy = 0;
#pragma unroll
                        for (int w = W - 1; w >= 0; --w) if (R[w]) wy = w;
                        y = wy * 64 + __builtin_ctzll(R[wy]);
#pragma unroll
                        for (int w = 0; w < W; ++w) if (w == wy) R[w] &= R[w] - 1;
                        if (rule1 && M.col[y] < l - 1) {
#pragma unroll
                            for (int w = 0; w < W; ++w) R[w] = 0;
                            continue;
                        }
                        break;
                    }
                    // next x in P after x
                    int nx = -1;
#pragma unroll
                    for (int w = W - 1; w >= 0; --w) {
                        uint64_t b = P[w] & (x < 0 ? ~0ull : upper_mask(x, w));
                        if (b) nx = w * 64 + __builtin_ctzll(b);
                    }
                    if (nx < 0 || (rule1 && M.col[nx] < l)) { done = true; break; }
                    x = nx;
#pragma unroll
                    for (int w = 0; w < W; ++w) R[w] = P[w] & M.rows[x][w] & upper_mask(x, w);
                }
                if (done) {
                    --sp;
                    continue;
                }
                if (lane == 0 || sp - 1 >= MAX_FRAMES) {
#pragma unroll
                    for (int w = 0; w < W; ++w) F.R[w] = R[w];
                    F.x = x;
                }
                wave_sync();
                uint64_t Pc[W];
#pragma unroll
                for (int w = 0; w < W; ++w) Pc[w] = R[w] & M.rows[y][w] & upper_mask(y, w);
                int lc = l - 2;
                if (work) wk_ops += W;
                if (popcW(Pc) < lc) continue;
                if (work && rule2 && lc >= 3) wk_ops += W;
                if (rule2 && lc >= 3 && distinct_colours(L, Pc) < lc) continue;
                node(Pc, lc, x, y);
            }
        }
    seed_done:
        if (!LIST) {
            if (sacc.hi) atomicOr(a.err, ERR_OVERFLOW);
            if (a.per_seed && lane == 0) a.per_seed[oi] = sacc.lo;
            uint64_t o = acc.lo;
            acc.lo += sacc.lo;
            if (acc.lo < o) ++acc.hi;
            acc.hi += sacc.hi;
        }
        wave_sync();
    }
    if (work && lane == 0) {
        atomicAdd(&a.work[0], (unsigned long long)wk_seeds);
        atomicAdd(&a.work[1], (unsigned long long)wk_nodes);
        atomicAdd(&a.work[2], (unsigned long long)wk_ops);
    }
    if (!LIST && lane == 0 && (acc.lo || acc.hi)) {
        unsigned long long old = atomicAdd(&a.total[0], (unsigned long long)acc.lo);
        unsigned long long carry = (old + acc.lo < old) ? 1ull : 0ull;
        if (acc.hi + carry) atomicAdd(&a.total[1], (unsigned long long)(acc.hi + carry));
    }
}

// |V(g_i)| of every edge: the candidate step of the branch kernel alone,
// one wave per edge.
__global__ void k_subsize(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const int32_t* __restrict__ erank, const int2* __restrict__ rrow,
                          const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                          const int32_t* __restrict__ rank, int64_t m, int32_t* __restrict__ out) {
    const int lane = lane_id();
    int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    int64_t nw = (int64_t)gridDim.x * blockDim.x / 64;
    for (int64_t e = wid; e < m; e += nw) {
        int32_t u = eu[e], v = ev[e], r = rank[e];
        int lo = rp[u], hi = rp[u + 1];
        while (lo < hi) { int mid = (lo + hi) >> 1; if (rrow[mid].y > r) lo = mid + 1; else hi = mid; }
        int lu = lo - rp[u];
        lo = rp[v]; hi = rp[v + 1];
        while (lo < hi) { int mid = (lo + hi) >> 1; if (rrow[mid].y > r) lo = mid + 1; else hi = mid; }
        int lv = lo - rp[v];
        int32_t xs = lu <= lv ? u : v, ys = lu <= lv ? v : u;
        int lx = lu <= lv ? lu : lv, c = 0;
        for (int base = 0; base < lx; base += 64) {
            int idx = base + lane;
            bool ok = false;
            if (idx < lx) {
                int32_t w = rrow[rp[xs] + idx].x;
                int q = lower_bound_i32(ci, rp[ys], rp[ys + 1], w);
                ok = q < rp[ys + 1] && ci[q] == w && erank[q] > r;
            }
            c += popc64(ballot(ok));
        }
        if (lane == 0) out[e] = c;
    }
}

namespace {

// persistent grid: resident blocks per CU times CUs, no more than the seeds need
template <int W, bool LIST>
int64_t grid_blocks(int64_t nseeds, int cus, int blocks_per_cu) {
    auto kern = k_branch<W, LIST>;
    size_t smem = 4 * sizeof(WaveMem<W>);
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess)
        return -1;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, smem) != hipSuccess) return -1;
    if (occ < 1) occ = 1;
    if (blocks_per_cu > 0 && blocks_per_cu < occ) occ = blocks_per_cu;
    int64_t grid = (int64_t)occ * cus;
    int64_t need = (nseeds + 3) / 4;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    return grid;
}

template <int W, bool LIST>
hipError_t launch_branch(const BranchArgs& a, int cus, int blocks_per_cu, hipStream_t s) {
    auto kern = k_branch<W, LIST>;
    size_t smem = 4 * sizeof(WaveMem<W>);
    int64_t grid = grid_blocks<W, LIST>(a.nseeds, cus, blocks_per_cu);
    if (grid < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), smem, s, a);
    return hipGetLastError();
}

}  // namespace

size_t branch_frame_bytes(int W) {
    switch (W) {
        case 1: return sizeof(Frame<1>);
        case 2: return sizeof(Frame<2>);
        case 3: return sizeof(Frame<3>);
        case 4: return sizeof(Frame<4>);
    }
    return 0;
}

int64_t branch_grid_waves(int W, int64_t nseeds, int cus, int bpc) {
    int64_t b = -1;
    switch (W) {
        case 1: b = grid_blocks<1, false>(nseeds, cus, bpc); break;
        case 2: b = grid_blocks<2, false>(nseeds, cus, bpc); break;
        case 3: b = grid_blocks<3, false>(nseeds, cus, bpc); break;
        case 4: b = grid_blocks<4, false>(nseeds, cus, bpc); break;
    }
    return b < 0 ? -1 : 4 * b;
}

hipError_t launch_branch_class(int W, bool list, const BranchArgs& a, int cus, int bpc, hipStream_t s) {
    if (list) return hipErrorInvalidValue;
    switch (W) {
        case 1: return launch_branch<1, false>(a, cus, bpc, s);
        case 2: return launch_branch<2, false>(a, cus, bpc, s);
        case 3: return launch_branch<3, false>(a, cus, bpc, s);
        case 4: return launch_branch<4, false>(a, cus, bpc, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_binom_init(hipStream_t s) {
    hipLaunchKernelGGL(k_binom_init, dim3((BIN_N + 255) / 256), dim3(256), 0, s);
    return hipGetLastError();
}

hipError_t launch_subsize(const int32_t* rp, const int32_t* ci, const int32_t* erank, const int2* rrow,
                          const int32_t* eu, const int32_t* ev, const int32_t* rank, int64_t m, int32_t* out,
                          hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_subsize, dim3(8192), dim3(256), 0, s, rp, ci, erank, rrow, eu, ev, rank, m, out);
    return hipGetLastError();
}

}  // namespace ebb
