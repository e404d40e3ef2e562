// handle.h -- the prepared graph held on the device, and internal entry
// points shared by the host-side files of libebbkc.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/ebbkc.h"

// Sub-branches of the node-parallel VBBkC roots (one slot per vertex with a
// non-empty N+(v), in position order); swapped with the edge arena while a
// count runs on them.
struct VertexArena {
    bool built = false;
    int64_t nseeds = 0;
    int32_t* seed_v = nullptr;     // vertex of each slot
    int32_t* seed_c = nullptr;     // |N+(v)|
    int32_t* seed_rthr = nullptr;  // rank of v's first out-edge minus one
    int64_t* row_off = nullptr;
    int64_t* vtx_off = nullptr;
    uint64_t* rows = nullptr;
    int32_t* gid = nullptr;
    int16_t* col = nullptr;
    uint64_t* nedges = nullptr;
    std::vector<int32_t> rank_host;  // rank of each slot's first out-edge (ascending)
    int64_t bytes = 0;
};

struct ebbkc_graph {
    int device = 0;
    int32_t n = 0;
    int64_t m = 0, nnz = 0;
    int32_t tau = 0, rounds = 0, max_degree = 0;
    double prepare_ms = 0.0;
    ebbkc_options opt{};
    int cu_count = 256;

    // id-sorted CSR (input copy) and per-entry edge rank
    int32_t* rp = nullptr;    // n+1
    int32_t* ci = nullptr;    // nnz
    int32_t* erank = nullptr; // nnz: rank of the edge of each entry
    // per edge (id order)
    int32_t* eu = nullptr;    // m, smaller endpoint
    int32_t* ev = nullptr;    // m, larger endpoint
    int32_t* sup0 = nullptr;  // m, common neighbours in G
    int32_t* rank = nullptr;  // m, position in pi_tau
    int32_t* level = nullptr; // m, truss level
    // full rows sorted by edge rank, descending: (neighbour, rank)
    int2* rrow = nullptr;     // nnz (row offsets = rp)
    // degree-oriented rows sorted by edge rank, descending: (neighbour, rank)
    int32_t* orp = nullptr;   // n+1
    int2* orow = nullptr;     // m
    int32_t* byrank = nullptr; // m: edge id at each rank
    // adjacency bitmap (n <= the adjacency bound): n rows of adjw words, and
    // per word the entries of the id-sorted row below it
    uint64_t* adj = nullptr;
    uint16_t* acum = nullptr;
    int32_t adjw = 0;
    int32_t* subsize = nullptr; // m: |V(g_i)| per edge (filled on demand)
    int32_t* vpos = nullptr;    // n: position in the root vertex order (orderings COLOR, DEGEN_VERTEX)
    int32_t* vcol = nullptr;    // n: greedy colour of G (ordering COLOR)
    bool subsize_ready = false;

    // sub-branch arena (built on the first count with k >= 4)
    bool arena_built = false;
    int64_t nseeds = 0;          // edges with |V(g_i)| >= 2, in rank order
    int32_t* seed_eid = nullptr;
    int32_t* seed_c = nullptr;
    int64_t* row_off = nullptr;
    int64_t* vtx_off = nullptr;
    uint64_t* arows = nullptr;
    int32_t* agid = nullptr;
    int16_t* acol = nullptr;
    uint64_t* nedges = nullptr;
    int64_t arena_bytes = 0;
    std::vector<int32_t> seed_rank_host; // rank of each slot (ascending)
    std::vector<int32_t> seed_c_host;    // |V(g_i)| of each slot (filled on demand)
    std::vector<int32_t> rank_host;      // rank of each edge (filled on demand)
    double arena_ms = 0.0;

    // per-call scratch (grown on demand, freed by destroy)
    void* scratch = nullptr;
    int32_t* rho_slab = nullptr;      // edge-rank matrices of the EBBkC-T search (allocated on first use)
    VertexArena varena;               // node-parallel VBBkC roots (built on first use)
    bool np_active = false;           // the vertex arena is swapped in
    size_t scratch_bytes = 0;
    uint64_t* d_counters = nullptr;   // small device counters
    uint64_t* h_counters = nullptr;   // pinned mirror
    double last_ms[4] = {0, 0, 0, 0};
    uint64_t last_work[4] = {0, 0, 0, 0};
    uint64_t last_work_class[4][4] = {};
    uint64_t last_total[2] = {0, 0};  // the last count, 128 bits
    bool last_total_ovf = false;      // it reached 2^128
    int64_t device_bytes = 0;
};

namespace ebb {
ebbkc_status prepare_impl(ebbkc_graph* g, const int32_t* row_ptr, const int32_t* col_idx, int32_t ptr_kind,
                          hipStream_t s);
ebbkc_status count_impl(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, const int64_t* d_eids,
                        int64_t ne, uint64_t* d_per_seed, uint64_t* out, hipStream_t s);
ebbkc_status list_impl(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, int32_t* d_buf, uint64_t cap,
                       uint32_t flags, uint64_t* out_written, uint64_t* out_checksums, hipStream_t s);
ebbkc_status subsize_impl(ebbkc_graph* g, hipStream_t s);
ebbkc_status arena_impl(ebbkc_graph* g, hipStream_t s);
hipError_t ensure_tables(int dev, hipStream_t s);
ebbkc_status count_seeds_impl(ebbkc_graph* g, int32_t k, const int64_t* eids, int64_t ne, int32_t ptr_kind,
                              uint64_t* out, hipStream_t s);
void* scratch_get(ebbkc_graph* g, size_t bytes);
ebbkc_status count_noalloc_impl(ebbkc_graph* g, int32_t k, uint64_t* out, hipStream_t s);
}  // namespace ebb
