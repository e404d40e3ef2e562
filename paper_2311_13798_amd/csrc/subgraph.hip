// subgraph.hip -- sub-branch construction into the arena (one wavefront per
// seed edge) and the |V(g_i)| of every edge.
//
// Each g_i is built in LDS by build_subbranch (build.h: candidates, the
// bitmap of the edges among them ranked after the seed, greedy colouring),
// then written to the seed's arena slot with its vertices in the order of
// Algorithm EBBkC-H (non-increasing colour, ties to the smaller vertex id):
// symmetric rows, colours and global ids.  The search kernels orient the rows
// low -> high.
#include "build.h"

namespace ebb {
namespace {

template <int W>
struct BuildMem {
    uint64_t rows[64 * W][W];
    int16_t col[64 * W];
    alignas(4) unsigned char work[build_scratch_bytes<W>()];
};

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
            if (idx < lx) ok = later_edge(G, ys, G.rrow[G.rp[xs] + idx].x, r);
            c += popc64(ballot(ok));
        }
        if (lane == 0) out[e] = c;
    }
}

template <int W>
__global__ __launch_bounds__(256) void k_build(BuildArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    BuildMem<W>& M = reinterpret_cast<BuildMem<W>*>(smem_raw)[threadIdx.x / 64];
    const BuildScratch<W> S = BuildScratch<W>::carve(M.work);
    const int lane = lane_id();
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
        uint32_t twoE = 0;
        const int c = build_subbranch<W>(G, u, v, r, a.seed_c[s], a.vcol, M.rows, M.col, S, &twoE);
        if (c < 0) {
            if (lane == 0) atomicOr(a.err, ERR_WIDTH);
            continue;
        }
        // relabel by colour desc, id asc, and write the slot
        int npos[W];
        order_positions<W>(c, M.col, S, npos);
        const int64_t ro = a.row_off[s], vo = a.vtx_off[s];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int i = lane + 64 * q;
            if (i < c) {
                uint64_t nr[W];
                relabelled_row<W>(M.rows, i, S, nr);
                uint64_t* dst = a.rows + ro + (int64_t)npos[q] * W;
#pragma unroll
                for (int w = 0; w < W; ++w) dst[w] = nr[w];
                a.gid[vo + npos[q]] = S.gid[i];
                a.col[vo + npos[q]] = M.col[i];
            }
        }
        if (lane == 0) a.nedges[s] = twoE / 2;
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
