// device_util.h -- wave-level helpers for the bitmap kernels (wave64).
#pragma once
#include "common.h"

namespace ebb {

// Order this wave's LDS accesses: everything before is visible to every lane after.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a wave-uniform 64-bit value in scalar registers
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// bits strictly above x within word w of a multi-word row
__device__ __forceinline__ uint64_t upper_mask(int x, int w) {
    int xw = x >> 6, xb = x & 63;
    if (w < xw) return 0;
    if (w > xw) return ~0ull;
    return xb == 63 ? 0ull : (~0ull << (xb + 1));
}

template <int W>
__device__ __forceinline__ int popcW(const uint64_t (&p)[W]) {
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) c += popc64(p[w]);
    return c;
}

// rows [0, c) as a W-word mask
template <int W>
__device__ __forceinline__ void prefix_mask(int c, uint64_t (&p)[W]) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
        int lo = 64 * w;
        p[w] = c >= lo + 64 ? ~0ull : (c > lo ? ((1ull << (c - lo)) - 1) : 0ull);
    }
}

}  // namespace ebb
