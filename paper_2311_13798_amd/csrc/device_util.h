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

// Wave64 reductions of 32-bit values: DPP moves within each row of 16 lanes
// (swap neighbours, swap pairs, mirror within 8, mirror within 16), then the
// four row results read into scalars.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
enum : int { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140 };

__device__ __forceinline__ uint32_t wsum_u32(uint32_t v) {
    int x = (int)v;
    x += dpp_mov<DPP_XOR1>(x);
    x += dpp_mov<DPP_XOR2>(x);
    x += dpp_mov<DPP_HALF_MIRROR>(x);
    x += dpp_mov<DPP_MIRROR>(x);
    return (uint32_t)__builtin_amdgcn_readlane(x, 0) + (uint32_t)__builtin_amdgcn_readlane(x, 16) +
           (uint32_t)__builtin_amdgcn_readlane(x, 32) + (uint32_t)__builtin_amdgcn_readlane(x, 48);
}

__device__ __forceinline__ int wmax_i32(int x) {
    x = max(x, dpp_mov<DPP_XOR1>(x));
    x = max(x, dpp_mov<DPP_XOR2>(x));
    x = max(x, dpp_mov<DPP_HALF_MIRROR>(x));
    x = max(x, dpp_mov<DPP_MIRROR>(x));
    return max(max(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
               max(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

__device__ __forceinline__ int wmin_i32(int x) {
    x = min(x, dpp_mov<DPP_XOR1>(x));
    x = min(x, dpp_mov<DPP_XOR2>(x));
    x = min(x, dpp_mov<DPP_HALF_MIRROR>(x));
    x = min(x, dpp_mov<DPP_MIRROR>(x));
    return min(min(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
               min(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

// bits strictly above x within word w of a multi-word row
__device__ __forceinline__ uint64_t upper_mask(int x, int w) {
    int xw = x >> 6, xb = x & 63;
    if (w < xw) return 0;
    if (w > xw) return ~0ull;
    return xb == 63 ? 0ull : (~0ull << (xb + 1));
}

// Pair u of the r(r-1)/2 pairs (i, j), i < j < r, numbered row by row (row i
// starts at i (2r - i - 1) / 2): the row from the quadratic's root, then
// corrected by whole rows against float rounding.
__device__ __forceinline__ void upper_pair(int u, int r, int& i, int& j) {
    const float R2 = 2.0f * (float)r - 1.0f;
    int ii = (int)((R2 - sqrtf(R2 * R2 - 8.0f * (float)u)) * 0.5f);
    ii = ii < 0 ? 0 : (ii > r - 2 ? r - 2 : ii);
    while (ii < r - 2 && (ii + 1) * (2 * r - ii - 2) / 2 <= u) ++ii;
    while (ii > 0 && ii * (2 * r - ii - 1) / 2 > u) --ii;
    i = ii;
    j = u - ii * (2 * r - ii - 1) / 2 + ii + 1;
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
