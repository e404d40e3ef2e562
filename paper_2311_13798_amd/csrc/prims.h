// prims.h -- device-wide primitives used by the EBBkC pipeline: exclusive
// scan, ordered compaction and a stable LSD radix sort of 64-bit keys.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebb {

// Exclusive prefix sum of in[0..n) into out[0..n) (int64).  If d_total is
// non-null the sum of all inputs is written there.  tmp must hold
// scan_tmp_elems(n) int64 values.
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan_i32(const int32_t* in, int64_t* out, int64_t n, int64_t* d_total, int64_t* tmp,
                              hipStream_t s);
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* d_total, int64_t* tmp,
                              hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).
// keys/vals are sorted in place; keys_alt/vals_alt are same-sized scratch;
// hist must hold radix_hist_elems(n) int64 values and tmp scan_tmp_elems of
// that.  vals may be null (keys only).
int64_t radix_hist_elems(int64_t n);
hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                          int bits, int64_t* hist, int64_t* tmp, hipStream_t s);

}  // namespace ebb
