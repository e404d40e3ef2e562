// list.hip -- k-clique listing: the search of Algorithm EBBkC-C_Rec with the
// outputs of its terminations (l = 1: S with each vertex; l = 2: S with each
// edge) written as tuples, plus tuple canonicalisation, lexicographic sorting
// and the listing checksums.  Up to k = 8 a tuple is sorted in registers and
// hashed as it is written, so no separate canonicalisation or checksum pass
// reads the buffer again (unless it is sorted afterwards).
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

// SplitMix64 output function (the tuple hash of the listing checksums)
__device__ __forceinline__ uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A tuple of at most 8 ids: the node's prefix pre[0..npre) (INT32_MAX
// beyond) with the leaf ids a (and b when two) inserted, sorted ascending,
// written at out[idx * k], its hash folded into the [ordered, unordered] sums.
__device__ __forceinline__ void put_tuple8(int32_t* __restrict__ out, int k, const int32_t (&pre)[8], int npre,
                                           int32_t a, int32_t b, bool two, uint64_t idx, uint64_t& ho,
                                           uint64_t& hu) {
    int32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = j == npre ? a : (two && j == npre + 1 ? b : pre[j]);
    sort_net<8>(v);
    int32_t* t = out + idx * (uint64_t)k;
    uint64_t h = (uint64_t)k;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < k) {
            t[j] = v[j];
            h = sm64(h ^ (uint64_t)(uint32_t)v[j]);
        }
    hu += h;
    ho += sm64(h ^ sm64(idx));
}

template <int W>
struct ListMem {
    uint64_t rows[64 * W][W];
    int32_t gid[64 * W];
    int32_t eoff[64 * W + 1];  // first tuple of each vertex's edges in the node being written
    // one-leaf tuples waiting to be sorted and hashed 64 at a time: buffer
    // index, leaf vertex and the pair (cx, cy) that reached their node
    uint64_t qidx[128];
    int16_t qz[128], qx[128], qy[128];
    int16_t col[64 * W];
    LFrame<W> fr[LIST_LDS_FRAMES];
};

// index of the j-th set bit (from 0) of x, which has more than j set bits
__device__ __forceinline__ int select_bit(uint64_t x, int j) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = x & ((1ull << w) - 1);
        const int c = __popcll(low);
        if (j >= c) {
            j -= c;
            x >>= w;
            pos += w;
        }
    }
    return pos;
}

}  // namespace

template <int W, bool FUSED>
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
    constexpr bool fused = FUSED;  // k <= 8
    uint64_t ho = 0, hu = 0;

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
        // the same prefix as register values (k <= 8, so at most one frame)
        auto prefix8 = [&](int32_t (&pre)[8], int depth, int cx, int cy) {
            int32_t f0 = INT32_MAX, f1 = INT32_MAX, c0 = INT32_MAX, c1 = INT32_MAX;
            if (depth > 0) {  // frame 0 always lives in LDS
                f0 = M.gid[M.fr[0].x];
                f1 = M.gid[M.fr[0].y];
            }
            if (cx >= 0) {
                c0 = M.gid[cx];
                c1 = M.gid[cy];
            }
            const int oc = 2 + 2 * depth;  // where (cx, cy) go
#pragma unroll
            for (int j = 0; j < 8; ++j)
                pre[j] = j == 0 ? su : j == 1 ? sv : (depth > 0 && j == 2) ? f0 : (depth > 0 && j == 3) ? f1
                       : (cx >= 0 && j == oc) ? c0 : (cx >= 0 && j == oc + 1) ? c1 : INT32_MAX;
            return oc + (cx >= 0 ? 2 : 0);
        };
        // queued one-leaf tuples (fused): 64 at a time, or all of them before
        // the frames their prefixes read change
        int qn = 0;
        auto flush1 = [&](bool all) {
            while (qn >= 64 || (all && qn > 0)) {
                const int take = qn < 64 ? qn : 64;
                if (lane < take) {
                    int32_t pre[8];
                    const int npre = prefix8(pre, sp, M.qx[lane], M.qy[lane]);
                    put_tuple8(a.out, k, pre, npre, M.gid[M.qz[lane]], 0, false, M.qidx[lane], ho, hu);
                }
                wave_sync();
                for (int i = take + lane; i < qn; i += 64) {  // entries [64, qn) move to [0, qn - 64)
                    M.qidx[i - take] = M.qidx[i];
                    M.qz[i - take] = M.qz[i];
                    M.qx[i - take] = M.qx[i];
                    M.qy[i - take] = M.qy[i];
                }
                wave_sync();
                qn -= take;
            }
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
                    const uint64_t idx = base + popc64(mk & lanemask_lt());
                    if constexpr (fused) {
                        const int e = qn + popc64(mk & lanemask_lt());
                        M.qidx[e] = idx;
                        M.qz[e] = (int16_t)(lane + 64 * q);
                        M.qx[e] = (int16_t)cx;
                        M.qy[e] = (int16_t)cy;
                    } else {
                        int32_t* t = a.out + idx * (uint64_t)k;
                        const int o = prefix(t, sp, cx, cy);
                        t[o] = M.gid[lane + 64 * q];
                    }
                }
                base += popc64(mk);
                if constexpr (fused) {
                    qn += popc64(mk);
                    wave_sync();
                    flush1(false);
                }
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
            if constexpr (fused) {
                // every lane takes every 64th tuple: vertex z from the edge
                // offsets, its other end the matching set bit of z's edge mask
                int32_t pre[8];
                const int npre = prefix8(pre, sp, cx, cy);
                uint32_t run = 0;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t inc = wave_incl_scan(cnt[q]);
                    M.eoff[lane + 64 * q] = (int32_t)(run + inc - cnt[q]);
                    run += __shfl(inc, 63, 64);
                }
                if (lane == 0) M.eoff[64 * W] = (int32_t)run;
                wave_sync();
                for (uint32_t t0 = 0; t0 < (uint32_t)tot; t0 += 64) {
                    const int t = (int)t0 + lane;
                    if (t < (int)tot) {
                        int lo = 0, hi = 64 * W;  // last z with eoff[z] <= t
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (M.eoff[mid] <= t) lo = mid; else hi = mid;
                        }
                        const int z = lo;
                        int j = t - M.eoff[z], w2 = -1;
#pragma unroll
                        for (int wy = 0; wy < W; ++wy) {
                            const uint64_t bits = P[wy] & M.rows[z][wy] & upper_mask(z, wy);
                            const int c = popc64(bits);
                            if (w2 < 0 && j < c) w2 = wy * 64 + select_bit(bits, j);
                            j -= c;
                        }
                        put_tuple8(a.out, k, pre, npre, M.gid[z], M.gid[w2], true, base + (uint64_t)t, ho, hu);
                    }
                }
                wave_sync();
                pos += tot;
                return;
            }
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
                    if constexpr (fused) flush1(true);
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
                if constexpr (fused) flush1(true);
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
        if constexpr (fused) flush1(true);
        if (pos != end && lane == 0) atomicOr(a.err, ERR_CAP);
        wave_sync();
    }
    if (fused) {
        ho = wave_sum(ho);
        hu = wave_sum(hu);
        if (lane == 0) {
            atomicAdd(&a.list_checksums[0], (unsigned long long)ho);
            atomicAdd(&a.list_checksums[1], (unsigned long long)hu);
        }
    }
}

// ---------------------------------------------------------------- tuple utilities

namespace {


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

template <int W, bool FUSED>
hipError_t launch_list_w(const SearchArgs& a, int cus, hipStream_t s) {
    auto kern = k_list<W, FUSED>;
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
    const bool fused = a.list_checksums != nullptr;
    switch (W) {
        case 1: return fused ? launch_list_w<1, true>(a, cus, s) : launch_list_w<1, false>(a, cus, s);
        case 2: return fused ? launch_list_w<2, true>(a, cus, s) : launch_list_w<2, false>(a, cus, s);
        case 3: return fused ? launch_list_w<3, true>(a, cus, s) : launch_list_w<3, false>(a, cus, s);
        case 4: return fused ? launch_list_w<4, true>(a, cus, s) : launch_list_w<4, false>(a, cus, s);
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
