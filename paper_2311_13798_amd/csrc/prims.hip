// prims.hip -- exclusive scan and stable LSD radix sort (wave64, gfx950).
#include "common.h"
#include "prims.h"

namespace ebb {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* total) {
    __shared__ int64_t wsum[SCAN_BLOCK / EBB_WAVE];
    int lane = lane_id(), w = threadIdx.x / EBB_WAVE;
    int64_t inc = wave_incl_scan(v);
    if (lane == EBB_WAVE - 1) wsum[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < SCAN_BLOCK / EBB_WAVE; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

template <typename T>
__global__ void k_tile_sums(const T* __restrict__ in, int64_t n, int64_t* __restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t acc = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j * SCAN_BLOCK + threadIdx.x;
        if (i < n) acc += (int64_t)in[i];
    }
    acc = wave_sum(acc);
    __shared__ int64_t ws[SCAN_BLOCK / EBB_WAVE];
    if (lane_id() == 0) ws[threadIdx.x / EBB_WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int i = 0; i < SCAN_BLOCK / EBB_WAVE; ++i) t += ws[i];
        part[blockIdx.x] = t;
    }
}

// one block scans the tile sums in place (any count)
__global__ void k_scan_parts(int64_t* __restrict__ part, int64_t np, int64_t* __restrict__ d_total) {
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < np; base += SCAN_BLOCK) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < np ? part[i] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan(v, &tot);
        if (i < np) part[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && d_total) *d_total = carry;
}

template <typename T>
__global__ void k_tile_scan(const T* __restrict__ in, int64_t* __restrict__ out, int64_t n,
                            const int64_t* __restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // each thread owns SCAN_ITEMS consecutive elements
    int64_t first = base + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = first + j;
        v[j] = i < n ? (int64_t)in[i] : 0;
        s += v[j];
    }
    int64_t tot;
    int64_t ex = block_excl_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = first + j;
        if (i < n) out[i] = ex;
        ex += v[j];
    }
}

template <typename T>
hipError_t scan_impl(const T* in, int64_t* out, int64_t n, int64_t* d_total, int64_t* tmp, hipStream_t s) {
    if (n <= 0) {
        if (d_total) return hipMemsetAsync(d_total, 0, sizeof(int64_t), s);
        return hipSuccess;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(SCAN_BLOCK), 0, s, tmp, nb, d_total);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, n, tmp);
    return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_BLOCK = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;
constexpr int RS_WAVES = RS_BLOCK / EBB_WAVE;

__global__ void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift, int64_t nb,
                          int64_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int j = 0; j < RS_ITEMS; ++j) {
        int64_t i = base + j * RS_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                             uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n, int shift,
                             int64_t nb, const int64_t* __restrict__ off) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[RS_WAVES][256];
    const int tid = threadIdx.x, lane = lane_id(), w = tid / EBB_WAVE;
    run[tid] = 0;
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int j = 0; j < RS_ITEMS; ++j) {
        int64_t i = base + j * RS_BLOCK + tid;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        uint32_t val = (valid && vin) ? vin[i] : 0;
        int d = (int)((key >> shift) & 0xFF);
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = ballot(valid && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        int lrank = popc64(peers & lanemask_lt());
#pragma unroll
        for (int q = 0; q < RS_WAVES; ++q) wcnt[q][tid] = 0;
        __syncthreads();
        if (valid && lrank == 0) wcnt[w][d] = (uint32_t)popc64(peers);
        __syncthreads();
        if (valid) {
            uint32_t before = 0;
            for (int q = 0; q < w; ++q) before += wcnt[q][d];
            int64_t pos = off[(int64_t)d * nb + blockIdx.x] + run[d] + before + lrank;
            kout[pos] = key;
            if (vout) vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < RS_WAVES; ++q) add += wcnt[q][tid];
        run[tid] += add;
        __syncthreads();
    }
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t exclusive_scan_i32(const int32_t* in, int64_t* out, int64_t n, int64_t* d_total, int64_t* tmp,
                              hipStream_t s) {
    return scan_impl<int32_t>(in, out, n, d_total, tmp, s);
}
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* d_total, int64_t* tmp,
                              hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, d_total, tmp, s);
}

int64_t radix_hist_elems(int64_t n) { return 256 * ((n + RS_TILE - 1) / RS_TILE) + 1; }

hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                          int bits, int64_t* hist, int64_t* tmp, hipStream_t s) {
    if (n <= 1 || bits <= 0) return hipSuccess;
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    uint64_t *ka = keys, *kb = keys_alt;
    uint32_t *va = vals, *vb = vals ? vals_alt : nullptr;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = p * 8;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(RS_BLOCK), 0, s, ka, n, shift, nb, hist);
        hipError_t e = exclusive_scan_i64(hist, hist, 256 * nb, nullptr, tmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(RS_BLOCK), 0, s, ka, va, kb, vb, n, shift, nb,
                           hist);
        uint64_t* kt = ka; ka = kb; kb = kt;
        uint32_t* vt = va; va = vb; vb = vt;
    }
    if (passes & 1) {
        hipError_t e = hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        if (vals) e = hipMemcpyAsync(vals, va, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace ebb
