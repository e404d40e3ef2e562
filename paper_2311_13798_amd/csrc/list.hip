// list.hip -- k-clique listing: the search of Algorithm EBBkC-C_Rec with the
// outputs of its terminations (l = 1: S with each vertex; l = 2: S with each
// edge) written as tuples, plus tuple canonicalisation, lexicographic sorting
// and the listing checksums.
//
// Every task writes its cliques from the offset its count (same task, same
// search space) reserved, so the buffer is deterministic.  Pruning Rules (1)
// and (2) apply as in counting; nodes are expanded down to l <= 2.
#include "arena.h"
#include "device_util.h"
#include "prims.h"

namespace ebb {

namespace {

template <int W>
struct LFrame {
    uint64_t P[W];
    uint64_t R[W];
    int32_t x, l, y, pad;
};

constexpr int LIST_LDS_FRAMES = 16;

template <int W>
struct ListMem {
    uint64_t rows[64 * W][W];
    int32_t gid[64 * W];
    int16_t col[64 * W];
    LFrame<W> fr[LIST_LDS_FRAMES];
};

}  // namespace

template <int W>
__global__ __launch_bounds__(256) void k_list(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ListMem<W>& M = reinterpret_cast<ListMem<W>*>(smem_raw)[threadIdx.x / 64];
    LFrame<W>* gfr = a.gframes ? reinterpret_cast<LFrame<W>*>(a.gframes) +
                                     ((int64_t)blockIdx.x * 4 + threadIdx.x / 64) * GLOBAL_FRAMES
                               : nullptr;
    auto FR = [&](int d) -> LFrame<W>& { return d < LIST_LDS_FRAMES ? M.fr[d] : gfr[d - LIST_LDS_FRAMES]; };
    const int lane = lane_id();
    const int k = a.k, opts = a.opts;
    const bool rule1 = opts & OPT_RULE1, rule2 = opts & OPT_RULE2;

    for (;;) {
        unsigned long long it = 0;
        if (lane == 0) it = atomicAdd(a.next, 1ull);
        it = uni64(__shfl(it, 0, 64));
        if ((int64_t)it >= a.ntasks) break;
        const int64_t task = a.tasks[it];
        const int64_t slot = task_slot(task);
        const int x0 = task_x0(task), x1 = task_x1(task);
        const int c = uniform_i32(a.A.seed_c[slot]);
        const int64_t ro = a.A.row_off[slot], vo = a.A.vtx_off[slot];
        const int32_t e = a.A.seed_eid[slot];
        const int32_t su = a.eu[e], sv = a.ev[e];
        for (int i = lane; i < c * W; i += 64) (&M.rows[0][0])[i] = a.A.rows[ro + i];
        for (int i = lane; i < c; i += 64) {
            M.col[i] = a.A.col[vo + i];
            M.gid[i] = a.A.gid[vo + i];
        }
        wave_sync();
        // [pos, end): this task's slots in the output
        uint64_t pos = a.task_off[it];
        const uint64_t end = pos + a.per_task[it];
        int sp = 0;

        // Write the tuples S + {x, y} + leaf, S = seed ends and the frames' pairs.
        // n_emit tuples; lane-owned leaf parts come from `leaf(i, t)`.
        auto prefix = [&](int32_t* t, int depth, int cx, int cy) {
            t[0] = su;
            t[1] = sv;
            int o = 2;
            for (int d = 0; d < depth; ++d) {
                const LFrame<W>& F = FR(d);
                t[o++] = M.gid[F.x];
                t[o++] = M.gid[F.y];
            }
            if (cx >= 0) {
                t[o++] = M.gid[cx];
                t[o++] = M.gid[cy];
            }
            return o;
        };
        // l = 1 node P reached through (cx, cy) at depth sp: S + {z}
        auto emit1 = [&](const uint64_t (&P)[W], int cx, int cy) {
            const int n = popcW(P);
            if (pos + n > end) { if (lane == 0) atomicOr(a.err, ERR_CAP); pos += n; return; }
            uint64_t base = pos;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const bool in = (P[q] >> lane) & 1;
                const uint64_t mk = ballot(in);
                if (in) {
                    int32_t* t = a.out + (base + popc64(mk & lanemask_lt())) * (uint64_t)k;
                    const int o = prefix(t, sp, cx, cy);
                    t[o] = M.gid[lane + 64 * q];
                }
                base += popc64(mk);
            }
            pos += n;
        };
        // l = 2 node P: S + {z, w} for every DAG edge z -> w inside P
        auto emit2 = [&](const uint64_t (&P)[W], int cx, int cy) {
            uint32_t cnt[W];
            uint64_t tot = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int z = lane + 64 * q;
                cnt[q] = 0;
                if ((P[q] >> lane) & 1) {
#pragma unroll
                    for (int w = 0; w < W; ++w) cnt[q] += popc64(P[w] & M.rows[z][w] & upper_mask(z, w));
                }
                tot += wave_sum(cnt[q]);
            }
            if (pos + tot > end) { if (lane == 0) atomicOr(a.err, ERR_CAP); pos += tot; return; }
            uint64_t base = pos;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const uint32_t inc = wave_incl_scan(cnt[q]);
                uint64_t my = base + inc - cnt[q];
                if (cnt[q]) {
                    const int z = lane + 64 * q;
#pragma unroll
                    for (int wy = 0; wy < W; ++wy) {
                        uint64_t bits = P[wy] & M.rows[z][wy] & upper_mask(z, wy);
                        while (bits) {
                            const int w2 = wy * 64 + __builtin_ctzll(bits);
                            bits &= bits - 1;
                            int32_t* t = a.out + my * (uint64_t)k;
                            const int o = prefix(t, sp, cx, cy);
                            t[o] = M.gid[z];
                            t[o + 1] = M.gid[w2];
                            ++my;
                        }
                    }
                }
                base += __shfl(inc, 63, 64);
            }
            pos += tot;
        };

        const int l0 = k - 2;
        uint64_t P0[W];
        prefix_mask<W>(c, P0);
        if (l0 == 1) {
            emit1(P0, -1, -1);
        } else if (l0 == 2) {
            emit2(P0, -1, -1);
        } else {
            uint64_t P[W], R[W];
            int x = x0 - 1, l = l0;
#pragma unroll
            for (int w = 0; w < W; ++w) { P[w] = P0[w]; R[w] = 0; }
            while (true) {
                int y = -1;
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
                    int nx = -1;
#pragma unroll
                    for (int w = W - 1; w >= 0; --w) {
                        const uint64_t b = P[w] & (x < 0 ? ~0ull : upper_mask(x, w));
                        if (b) nx = w * 64 + __builtin_ctzll(b);
                    }
                    const int xlim = sp == 0 ? x1 : c;
                    if (nx < 0 || nx >= xlim || (rule1 && M.col[nx] < l)) { y = -1; break; }
                    x = nx;
#pragma unroll
                    for (int w = 0; w < W; ++w) R[w] = P[w] & M.rows[x][w] & upper_mask(x, w);
                }
                if (y < 0) {
                    if (sp == 0) break;
                    --sp;
                    LFrame<W>& F = FR(sp);
#pragma unroll
                    for (int w = 0; w < W; ++w) { P[w] = uni64(F.P[w]); R[w] = uni64(F.R[w]); }
                    x = uniform_i32(F.x);
                    l = uniform_i32(F.l);
                    continue;
                }
                uint64_t Pc[W];
#pragma unroll
                for (int w = 0; w < W; ++w) Pc[w] = R[w] & M.rows[y][w] & upper_mask(y, w);
                const int lc = l - 2;
                if (popcW(Pc) < lc) continue;
                if (rule2 && lc >= 3) {
                    // distinct colours among Pc: count colour changes along Pc
                    int dc = 0, prev = -1;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        uint64_t b = Pc[w];
                        while (b && dc < lc) {
                            const int z = w * 64 + __builtin_ctzll(b);
                            b &= b - 1;
                            const int cz = M.col[z];
                            dc += cz != prev;
                            prev = cz;
                        }
                    }
                    if (dc < lc) continue;
                }
                if (lc == 1) { emit1(Pc, x, y); continue; }
                if (lc == 2) { emit2(Pc, x, y); continue; }
                if (sp >= LIST_LDS_FRAMES + (gfr ? GLOBAL_FRAMES : 0)) {
                    if (lane == 0) atomicOr(a.err, ERR_DEPTH);
                    continue;
                }
                if (lane == 0 || sp >= LIST_LDS_FRAMES) {
                    LFrame<W>& F = FR(sp);
#pragma unroll
                    for (int w = 0; w < W; ++w) { F.P[w] = P[w]; F.R[w] = R[w]; }
                    F.x = x;
                    F.l = l;
                    F.y = y;
                }
                ++sp;
                wave_sync();
#pragma unroll
                for (int w = 0; w < W; ++w) { P[w] = Pc[w]; R[w] = 0; }
                x = -1;
                l = lc;
            }
        }
        if (pos != end && lane == 0) atomicOr(a.err, ERR_CAP);
        wave_sync();
    }
}

// ---------------------------------------------------------------- tuple utilities

namespace {

template <int N>
__device__ __forceinline__ void sort_net(int32_t (&v)[N]) {
    // bitonic sorting network, ascending
#pragma unroll
    for (int size = 2; size <= N; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const int32_t a = v[i], b = v[j];
                    const bool sw = up ? (a > b) : (a < b);
                    v[i] = sw ? b : a;
                    v[j] = sw ? a : b;
                }
            }
}

template <int N>
__global__ void k_canon(int32_t* __restrict__ buf, int64_t n, int k) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v[N];
        int32_t* t = buf + i * k;
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = j < k ? t[j] : INT32_MAX;
        sort_net<N>(v);
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (j < k) t[j] = v[j];
    }
}

// keys of a column group for the permutation idx: concatenated columns [c0, c1)
__global__ void k_col_keys(const int32_t* __restrict__ buf, const uint32_t* __restrict__ idx, int64_t n, int k,
                           int c0, int c1, int bits, uint64_t* __restrict__ keys) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* t = buf + (int64_t)idx[i] * k;
        uint64_t key = 0;
        for (int c = c0; c < c1; ++c) key = (key << bits) | (uint64_t)(uint32_t)t[c];
        keys[i] = key;
    }
}

__global__ void k_iota_u32(uint32_t* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (uint32_t)i;
}

__global__ void k_gather_tuples(const int32_t* __restrict__ src, const uint32_t* __restrict__ idx, int64_t n, int k,
                                int32_t* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * k; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / k, c = i - r * k;
        dst[i] = src[(int64_t)idx[r] * k + c];
    }
}

__device__ __forceinline__ uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// [ordered, unordered] checksums (sums mod 2^64)
__global__ void k_checksums(const int32_t* __restrict__ buf, int64_t n, int k, unsigned long long* __restrict__ out) {
    uint64_t ho = 0, hu = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* t = buf + i * k;
        uint64_t h = (uint64_t)k;
        for (int j = 0; j < k; ++j) h = sm64(h ^ (uint64_t)(uint32_t)t[j]);
        hu += h;
        ho += sm64(h ^ sm64((uint64_t)i));
    }
    ho = wave_sum(ho);
    hu = wave_sum(hu);
    if (lane_id() == 0) {
        atomicAdd(&out[0], (unsigned long long)ho);
        atomicAdd(&out[1], (unsigned long long)hu);
    }
}

__global__ void k_list_small(const int32_t* __restrict__ byrank, const int32_t* __restrict__ eu,
                             const int32_t* __restrict__ ev, int64_t lo, int64_t hi, int k, int32_t* __restrict__ out) {
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (int64_t)gridDim.x * blockDim.x) {
        if (k == 1) {
            out[i - lo] = (int32_t)i;
        } else {
            const int32_t e = byrank[i];
            out[2 * (i - lo)] = eu[e];
            out[2 * (i - lo) + 1] = ev[e];
        }
    }
}

inline unsigned gridn(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (unsigned)b;
}

template <int W>
hipError_t launch_list_w(const SearchArgs& a, int cus, hipStream_t s) {
    auto kern = k_list<W>;
    const size_t smem = 4 * sizeof(ListMem<W>);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, smem);
    if (e != hipSuccess) return e;
    if (occ < 1) occ = 1;
    int64_t grid = (int64_t)occ * cus, need = (a.ntasks + 3) / 4;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), smem, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_list(int W, const SearchArgs& a, int cus, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    switch (W) {
        case 1: return launch_list_w<1>(a, cus, s);
        case 2: return launch_list_w<2>(a, cus, s);
        case 3: return launch_list_w<3>(a, cus, s);
        case 4: return launch_list_w<4>(a, cus, s);
    }
    return hipErrorInvalidValue;
}

size_t list_frame_bytes(int W) {
    switch (W) {
        case 1: return sizeof(LFrame<1>);
        case 2: return sizeof(LFrame<2>);
        case 3: return sizeof(LFrame<3>);
        case 4: return sizeof(LFrame<4>);
    }
    return 0;
}

int64_t list_grid_waves(int W, int64_t ntasks, int cus) {
    (void)W;
    // upper bound: eight blocks of four waves per CU
    int64_t g = 8 * (int64_t)cus, need = (ntasks + 3) / 4;
    return 4 * (g < need ? g : need);
}

hipError_t canon_tuples(int32_t* buf, int64_t n, int k, hipStream_t s) {
    if (n <= 0 || k <= 1) return hipSuccess;
    if (k <= 4) hipLaunchKernelGGL(k_canon<4>, dim3(gridn(n)), dim3(256), 0, s, buf, n, k);
    else if (k <= 8) hipLaunchKernelGGL(k_canon<8>, dim3(gridn(n)), dim3(256), 0, s, buf, n, k);
    else if (k <= 16) hipLaunchKernelGGL(k_canon<16>, dim3(gridn(n)), dim3(256), 0, s, buf, n, k);
    else if (k <= 32) hipLaunchKernelGGL(k_canon<32>, dim3(gridn(n)), dim3(256), 0, s, buf, n, k);
    else if (k <= 64) hipLaunchKernelGGL(k_canon<64>, dim3(gridn(n)), dim3(256), 0, s, buf, n, k);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// Lexicographic order of n tuples of k ids below 2^bits: LSD over groups of
// columns packed into 64-bit keys, then a gather.  tmp sizes: keys 2n
// (uint64), idx 2n (uint32), hist/htmp as radix_sort_u64, out n*k int32.
hipError_t sort_tuples(int32_t* buf, int64_t n, int k, int bits, uint64_t* keys, uint64_t* keys2, uint32_t* idx,
                       uint32_t* idx2, int64_t* hist, int64_t* htmp, int32_t* tmpbuf, hipStream_t s) {
    if (n <= 1) return hipSuccess;
    hipLaunchKernelGGL(k_iota_u32, dim3(gridn(n)), dim3(256), 0, s, idx, n);
    const int per = bits > 0 ? 64 / bits : k;
    int c1 = k;
    while (c1 > 0) {
        const int c0 = c1 - per > 0 ? c1 - per : 0;
        hipLaunchKernelGGL(k_col_keys, dim3(gridn(n)), dim3(256), 0, s, buf, idx, n, k, c0, c1, bits, keys);
        hipError_t e = radix_sort_u64(keys, idx, keys2, idx2, n, bits * (c1 - c0), hist, htmp, s);
        if (e != hipSuccess) return e;
        c1 = c0;
    }
    hipLaunchKernelGGL(k_gather_tuples, dim3(gridn(n * k)), dim3(256), 0, s, buf, idx, n, k, tmpbuf);
    hipError_t e = hipMemcpyAsync(buf, tmpbuf, sizeof(int32_t) * (size_t)(n * k), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t tuple_checksums(const int32_t* buf, int64_t n, int k, unsigned long long* d_out, hipStream_t s) {
    hipError_t e = hipMemsetAsync(d_out, 0, 2 * sizeof(uint64_t), s);
    if (e != hipSuccess) return e;
    if (n > 0) hipLaunchKernelGGL(k_checksums, dim3(gridn(n)), dim3(256), 0, s, buf, n, k, d_out);
    return hipGetLastError();
}

hipError_t list_small(const int32_t* byrank, const int32_t* eu, const int32_t* ev, int64_t lo, int64_t hi, int k,
                      int32_t* out, hipStream_t s) {
    if (hi > lo) hipLaunchKernelGGL(k_list_small, dim3(gridn(hi - lo)), dim3(256), 0, s, byrank, eu, ev, lo, hi, k, out);
    return hipGetLastError();
}

}  // namespace ebb
