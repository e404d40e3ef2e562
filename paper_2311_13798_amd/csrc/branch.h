// branch.h -- arguments of the EBBkC branch kernels (count and list modes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebb {

enum : int { ERR_WIDTH = 1, ERR_OVERFLOW = 2, ERR_DEPTH = 4, ERR_CAP = 8 };

enum : int { OPT_ET = 1, OPT_TPLEX2 = 2, OPT_RULE1 = 4, OPT_RULE2 = 8, OPT_WORK = 16 };

constexpr int MAX_FRAMES = 24;   // search frames kept in LDS (nodes with l >= 4)
constexpr int GLOBAL_FRAMES = 112; // further frames in device memory, per wave
constexpr int MAX_K = 2 + 2 * (MAX_FRAMES + GLOBAL_FRAMES) + 2;

struct BranchArgs {
    // prepared graph
    const int32_t* rp;
    const int32_t* ci;
    const int32_t* erank;
    const int2* rrow;
    const int32_t* orp;
    const int2* orow;
    const int32_t* eu;
    const int32_t* ev;
    const int32_t* rank;
    // seeds: edge ids; processed heaviest-first when reverse != 0
    const int32_t* seeds;
    int64_t nseeds;
    int32_t reverse;
    int32_t k;
    int32_t opts;
    int32_t pad;
    // where per-seed results go: index = out_base + (position in seeds), or
    // out_index[position] when out_index is set
    int64_t out_base;
    const int64_t* out_index;
    // outputs
    unsigned long long* next;   // work counter (zeroed by the host)
    unsigned long long* total;  // [lo, hi] 128-bit total
    uint64_t* per_seed;         // optional per-seed counts
    int* err;
    // listing
    const uint64_t* offsets;    // per-seed first output tuple (indexed like per_seed)
    int32_t* out;               // tuples of k int32
    uint64_t cap;
    unsigned long long* work;   // [seeds built, nodes, word ops] when OPT_WORK
    // deep-search frames (only needed when k > 2 + 2 * MAX_FRAMES + 2)
    void* gframes;              // GLOBAL_FRAMES frames per wave of the grid
};

size_t branch_frame_bytes(int W);
int64_t branch_grid_waves(int W, int64_t nseeds, int cus, int blocks_per_cu);

hipError_t launch_branch_class(int W, bool list, const BranchArgs& a, int cus, int blocks_per_cu, hipStream_t s);
hipError_t launch_binom_init(hipStream_t s);
hipError_t launch_subsize(const int32_t* rp, const int32_t* ci, const int32_t* erank, const int2* rrow,
                          const int32_t* eu, const int32_t* ev, const int32_t* rank, int64_t m, int32_t* out,
                          hipStream_t s);

}  // namespace ebb
