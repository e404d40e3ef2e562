// subgraph.hip -- sub-branch construction (one wavefront per seed edge).
//
// For a seed e_i = (u,v) of rank r (Eq. edge-oriented-branching):
//   1. candidates  V(g_i) = {w : (u,w) and (v,w) both ranked after e_i}.  The
//                  shorter of the two rank-sorted row prefixes (entries ranked
//                  after r) is scanned; each entry is looked up in the other
//                  endpoint's id-sorted row, whose rank must also exceed r.
//   2. sub-graph   E(g_i): pairs of V(g_i) joined by an edge ranked after r.
//                  Every member's degree-oriented row prefix ranked after r
//                  is scanned (all members' prefixes flattened over the
//                  wave's lanes) against an LDS hash of V(g_i); each such
//                  edge is met exactly once.
//   3. colouring   greedy colouring (colours 1, 2, ...) visiting vertices by
//                  non-increasing degree in g_i, ties to the smaller vertex
//                  id; then vertices are relabelled by non-increasing colour,
//                  ties to the smaller vertex id (Section 4.3; Algorithm
//                  EBBkC-H colours each g_i and orients it by this order).
//                  Under EBBkC-C the colours of G's own colouring are kept
//                  instead (renumbered 1..D among the colours present).
// The relabelled symmetric rows, colours and global ids go to the seed's
// arena slot; the search kernels orient them low -> high.
#include "arena.h"
#include "device_util.h"

namespace ebb {
namespace {

template <int W>
constexpr int hash_size() { return W <= 1 ? 128 : (W <= 2 ? 256 : 512); }

__device__ __forceinline__ uint32_t hslot(int32_t key, int hs) {
    return ((uint32_t)key * 2654435761u) & (uint32_t)(hs - 1);
}

template <int W>
struct BuildMem {
    uint64_t rows[64 * W][W];
    int32_t gid[64 * W];
    int32_t key[64 * W];
    int32_t hkey[hash_size<W>()];
    int16_t hval[hash_size<W>()];
    int16_t seq[64 * W];
    int16_t col[64 * W];
};

template <int W>
__device__ __forceinline__ int hash_find(const BuildMem<W>& M, int32_t key) {
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

}  // namespace

// |V(g_i)| of every edge: the candidate step alone, one wave per edge.
__global__ void k_subsize(GraphView G, int64_t m, int32_t* __restrict__ out) {
    const int lane = lane_id();
    int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    int64_t nw = (int64_t)gridDim.x * blockDim.x / 64;
    for (int64_t e = wid; e < m; e += nw) {
        const int32_t u = G.eu[e], v = G.ev[e], r = G.rank[e];
        const int lu = prefix_after(G.rp, G.rrow, u, r), lv = prefix_after(G.rp, G.rrow, v, r);
        const int32_t xs = lu <= lv ? u : v, ys = lu <= lv ? v : u;
        const int lx = lu <= lv ? lu : lv;
        int c = 0;
        for (int base = 0; base < lx; base += 64) {
            const int idx = base + lane;
            bool ok = false;
            if (idx < lx) {
                const int32_t w = G.rrow[G.rp[xs] + idx].x;
                const int q = lower_bound_i32(G.ci, G.rp[ys], G.rp[ys + 1], w);
                ok = q < G.rp[ys + 1] && G.ci[q] == w && G.erank[q] > r;
            }
            c += popc64(ballot(ok));
        }
        if (lane == 0) out[e] = c;
    }
}

template <int W>
__global__ __launch_bounds__(256) void k_build(BuildArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    BuildMem<W>& M = reinterpret_cast<BuildMem<W>*>(smem_raw)[threadIdx.x / 64];
    const int lane = lane_id();
    constexpr int CAP = 64 * W;
    constexpr int HS = hash_size<W>();
    const GraphView& G = a.G;

    for (;;) {
        unsigned long long it = 0;
        if (lane == 0) it = atomicAdd(a.next, 1ull);
        it = uni64(__shfl(it, 0, 64));
        if ((int64_t)it >= a.n) break;
        const int32_t s = a.list[it];
        const int32_t e = a.seed_eid[s];
        // a vertex slot is the edge slot with both ends at the vertex: its
        // row intersected with itself above the threshold is N+(v)
        const int32_t u = a.seed_rthr ? e : G.eu[e], v = a.seed_rthr ? e : G.ev[e];
        const int32_t r = a.seed_rthr ? a.seed_rthr[s] : G.rank[e];

        // ---- 1. candidates
        const int lu = prefix_after(G.rp, G.rrow, u, r), lv = prefix_after(G.rp, G.rrow, v, r);
        const int32_t xs = lu <= lv ? u : v, ys = lu <= lv ? v : u;
        const int lx = lu <= lv ? lu : lv;
        int c = 0;
        for (int base = 0; base < lx; base += 64) {
            const int idx = base + lane;
            bool ok = false;
            int32_t w = -1;
            if (idx < lx) {
                w = G.rrow[G.rp[xs] + idx].x;
                const int q = lower_bound_i32(G.ci, G.rp[ys], G.rp[ys + 1], w);
                ok = q < G.rp[ys + 1] && G.ci[q] == w && G.erank[q] > r;
            }
            const uint64_t mk = ballot(ok);
            if (ok) {
                const int p = c + popc64(mk & lanemask_lt());
                if (p < CAP) M.gid[p] = w;
            }
            c += popc64(mk);
        }
        c = uniform_i32(c);
        if (c > CAP || c != a.seed_c[s]) {
            if (lane == 0) atomicOr(a.err, ERR_WIDTH);
            continue;
        }

        // ---- 2. sub-graph bitmap
        for (int j = lane; j < HS; j += 64) M.hkey[j] = -1;
        for (int i = lane; i < c; i += 64)
#pragma unroll
            for (int w = 0; w < W; ++w) M.rows[i][w] = 0;
        wave_sync();
        for (int i = lane; i < c; i += 64) {
            const int32_t key = M.gid[i];
            uint32_t h = hslot(key, HS);
            while (true) {
                const int32_t old = atomicCAS(&M.hkey[h], -1, key);
                if (old == -1) { M.hval[h] = (int16_t)i; break; }
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
                    const int32_t w = M.gid[i];
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
                if (i < c) M.key[i] = total + inc - plen[q];
                total += __shfl(inc, 63, 64);
            }
            wave_sync();
            for (int base = 0; base < total; base += 64) {
                const int j = base + lane;
                if (j < total) {
                    int lo = 0, hi = c;  // last member whose offset is <= j
                    while (hi - lo > 1) {
                        int mid = (lo + hi) >> 1;
                        if (M.key[mid] <= j) lo = mid; else hi = mid;
                    }
                    const int i = lo;
                    const int2 yr = G.orow[G.orp[M.gid[i]] + (j - M.key[i])];
                    const int jj = hash_find(M, yr.x);
                    if (jj >= 0) {
                        atomicOr((unsigned long long*)&M.rows[i][jj >> 6], 1ull << (jj & 63));
                        atomicOr((unsigned long long*)&M.rows[jj][i >> 6], 1ull << (i & 63));
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
                for (int w = 0; w < W; ++w) d += popc64(M.rows[i][w]);
                M.key[i] = d;
                dsum += d;
            }
        }
        dsum = wave_sum(dsum);
        wave_sync();
        if (a.vcol) {
            // ---- 3'. G's colouring kept (EBBkC-C): the colours present are
            // renumbered 1..D in their order, which changes neither the order
            // below nor the number of colours in any vertex set
            for (int i = lane; i < c; i += 64) M.key[i] = a.vcol[M.gid[i]];
            wave_sync();
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int i = lane + 64 * q;
                const int ki = i < c ? M.key[i] : 0, gi = i < c ? M.gid[i] : 0;
                int ord = 0;
                for (int j = 0; j < c; ++j) {
                    const int kj = M.key[j], gj = M.gid[j];
                    ord += (kj > ki) || (kj == ki && gj < gi);
                }
                if (i < c) M.seq[ord] = (int16_t)i;
            }
            wave_sync();
            int cum[W];
            int starts = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int p = lane + 64 * q;
                const bool st = p < c && (p == 0 || M.key[M.seq[p]] != M.key[M.seq[p - 1]]);
                const uint64_t mk = ballot(st);
                cum[q] = starts + popc64(mk & (lanemask_lt() | (1ull << lane)));
                starts += popc64(mk);
            }
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int p = lane + 64 * q;
                if (p < c) M.col[M.seq[p]] = (int16_t)(starts - cum[q] + 1);
            }
            wave_sync();
        } else {
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int i = lane + 64 * q;
                const int di = i < c ? M.key[i] : 0, gi = i < c ? M.gid[i] : 0;
                int ord = 0;
                for (int j = 0; j < c; ++j) {
                    const int dj = M.key[j], gj = M.gid[j];
                    ord += (dj > di) || (dj == di && gj < gi);
                }
                if (i < c) M.seq[ord] = (int16_t)i;
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
                const int i = M.seq[t];
                uint64_t A[W];
#pragma unroll
                for (int w = 0; w < W; ++w) A[w] = M.rows[i][w];
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
                if (lane == 0) M.col[i] = (int16_t)(found + 1);
            }
            wave_sync();
        }
        // ---- 3c. relabel by colour desc, id asc, and write the slot
        int npos[W];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int i = lane + 64 * q;
            const int ci_ = i < c ? M.col[i] : 0, gi = i < c ? M.gid[i] : 0;
            int ord = 0;
            for (int j = 0; j < c; ++j) {
                const int cj = M.col[j], gj = M.gid[j];
                ord += (cj > ci_) || (cj == ci_ && gj < gi);
            }
            npos[q] = ord;
            if (i < c) M.key[i] = ord;
        }
        wave_sync();
        const int64_t ro = a.row_off[s], vo = a.vtx_off[s];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int i = lane + 64 * q;
            if (i < c) {
                uint64_t nr[W];
#pragma unroll
                for (int w = 0; w < W; ++w) nr[w] = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    uint64_t b = M.rows[i][w];
                    while (b) {
                        const int j = w * 64 + __builtin_ctzll(b);
                        b &= b - 1;
                        const int pj = M.key[j];
#pragma unroll
                        for (int ww = 0; ww < W; ++ww)
                            if (ww == (pj >> 6)) nr[ww] |= 1ull << (pj & 63);
                    }
                }
                uint64_t* dst = a.rows + ro + (int64_t)npos[q] * W;
#pragma unroll
                for (int w = 0; w < W; ++w) dst[w] = nr[w];
                a.gid[vo + npos[q]] = M.gid[i];
                a.col[vo + npos[q]] = M.col[i];
            }
        }
        if (lane == 0) a.nedges[s] = dsum / 2;
        wave_sync();
    }
}

namespace {
template <int W>
hipError_t launch_build_w(const BuildArgs& a, int cus, hipStream_t s) {
    auto kern = k_build<W>;
    const size_t smem = 4 * sizeof(BuildMem<W>);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, smem);
    if (e != hipSuccess) return e;
    if (occ < 1) occ = 1;
    int64_t grid = (int64_t)occ * cus, need = (a.n + 3) / 4;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), smem, s, a);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_build(int W, const BuildArgs& a, int cus, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    switch (W) {
        case 1: return launch_build_w<1>(a, cus, s);
        case 2: return launch_build_w<2>(a, cus, s);
        case 3: return launch_build_w<3>(a, cus, s);
        case 4: return launch_build_w<4>(a, cus, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_subsize(const GraphView& G, int64_t m, int32_t* out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_subsize, dim3(8192), dim3(256), 0, s, G, m, out);
    return hipGetLastError();
}

}  // namespace ebb
