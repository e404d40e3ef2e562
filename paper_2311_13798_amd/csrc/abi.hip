// abi.hip -- the extern "C" boundary of libebbkc (declared in include/ebbkc.h).
#include <new>

#include "arena.h"
#include "common.h"
#include "handle.h"

extern "C" {

void ebbkc_default_options(ebbkc_options* opt) {
    if (!opt) return;
    *opt = ebbkc_options{};
    opt->early_termination = 1;
    opt->t_plex = 0;
    opt->rule1 = 1;
    opt->rule2 = 1;
    opt->waves_per_block = 4;
    opt->blocks_per_cu = 0;
    opt->split_threshold = 0;
}

const char* ebbkc_strerror(ebbkc_status s) {
    switch (s) {
        case EBBKC_OK: return "ok";
        case EBBKC_E_INVALID_ARG: return "invalid argument";
        case EBBKC_E_BAD_CSR: return "input is not a simple undirected CSR with sorted rows";
        case EBBKC_E_OOM: return "device memory exhausted";
        case EBBKC_E_K_RANGE: return "k out of the supported range";
        case EBBKC_E_BUFFER_TOO_SMALL: return "listing buffer too small";
        case EBBKC_E_OVERFLOW: return "exact count does not fit 64 bits";
        case EBBKC_E_WIDTH: return "a sub-branch exceeds the widest bitmap class";
        case EBBKC_E_HIP: return "HIP runtime error";
        case EBBKC_E_CANCELLED: return "cancelled";
        case EBBKC_E_SCRATCH: return "the count needs more scratch than the fixed no-allocation buffer holds";
    }
    return "unknown status";
}

void ebbkc_destroy(ebbkc_graph* g) {
    if (!g) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    void* ptrs[] = {g->rp, g->ci, g->erank, g->eu, g->ev, g->sup0, g->rank, g->level, g->rrow, g->orp, g->orow,
                    g->byrank, g->subsize, g->scratch, g->d_counters, g->seed_eid, g->seed_c, g->row_off,
                    g->vtx_off, g->arows, g->agid, g->acol, g->nedges, g->vpos, g->vcol, g->rho_slab, g->adj, g->acum,
                    g->varena.seed_v, g->varena.seed_c, g->varena.seed_rthr, g->varena.row_off,
                    g->varena.vtx_off, g->varena.rows, g->varena.gid, g->varena.col, g->varena.nedges};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (g->h_counters) (void)hipHostFree(g->h_counters);
    (void)hipSetDevice(cur);
    delete g;
}

ebbkc_status ebbkc_prepare(const int32_t* row_ptr, const int32_t* col_idx, int32_t n, int64_t nnz, int32_t ptr_kind,
                           const ebbkc_options* opt, void* stream, ebbkc_graph** out) {
    if (!out || !row_ptr || n < 0 || nnz < 0 || (nnz > 0 && !col_idx)) return EBBKC_E_INVALID_ARG;
    if (ptr_kind != EBBKC_PTR_HOST && ptr_kind != EBBKC_PTR_DEVICE) return EBBKC_E_INVALID_ARG;
    if (nnz > 0x7fffffffLL) return EBBKC_E_INVALID_ARG;  // int32 row offsets
    ebbkc_graph* g = new (std::nothrow) ebbkc_graph();
    if (!g) return EBBKC_E_OOM;
    if (hipGetDevice(&g->device) != hipSuccess) { delete g; return EBBKC_E_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) != hipSuccess) { delete g; return EBBKC_E_HIP; }
    g->cu_count = prop.multiProcessorCount;
    if (opt) g->opt = *opt; else ebbkc_default_options(&g->opt);
    if (g->opt.ordering < EBBKC_ORDER_HYBRID || g->opt.ordering > EBBKC_ORDER_DEGEN_VERTEX_NP ||
        g->opt.batch_build < EBBKC_BATCH_AUTO || g->opt.batch_build > EBBKC_BATCH_BUILD || g->opt.node_split < -1 ||
        g->opt.t_plex < 0 || g->opt.t_plex > 16 || g->opt.adj_max_n < -1 || g->opt.adj_max_n > ebb::ADJ_MAX_N) {
        delete g;
        return EBBKC_E_INVALID_ARG;
    }
    g->n = n;
    g->nnz = nnz;
    ebbkc_status st = ebb::prepare_impl(g, row_ptr, col_idx, ptr_kind, (hipStream_t)stream);
    if (st != EBBKC_OK) { ebbkc_destroy(g); return st; }
    *out = g;
    return EBBKC_OK;
}

ebbkc_status ebbkc_count(ebbkc_graph* g, int32_t k, uint64_t* out_count, void* stream) {
    if (!g || !out_count) return EBBKC_E_INVALID_ARG;
    if (k < 1) return EBBKC_E_K_RANGE;
    if (k == 1) { *out_count = (uint64_t)g->n; return EBBKC_OK; }
    if (k == 2) { *out_count = (uint64_t)g->m; return EBBKC_OK; }
    if (k - 2 > g->tau) { *out_count = 0; return EBBKC_OK; }  // no sub-branch can hold k-2 vertices
    return ebb::count_impl(g, k, 0, g->m, nullptr, 0, nullptr, out_count, (hipStream_t)stream);
}

ebbkc_status ebbkc_count_noalloc(ebbkc_graph* g, int32_t k, uint64_t* out_count, void* stream) {
    if (!g || !out_count) return EBBKC_E_INVALID_ARG;
    if (k < 1) return EBBKC_E_K_RANGE;
    if (k == 1) { *out_count = (uint64_t)g->n; return EBBKC_OK; }
    if (k == 2) { *out_count = (uint64_t)g->m; return EBBKC_OK; }
    if (k - 2 > g->tau) { *out_count = 0; return EBBKC_OK; }
    return ebb::count_noalloc_impl(g, k, out_count, (hipStream_t)stream);
}

ebbkc_status ebbkc_count128(ebbkc_graph* g, int32_t k, uint64_t out_count[2], void* stream) {
    if (!g || !out_count) return EBBKC_E_INVALID_ARG;
    uint64_t lo = 0;
    ebbkc_status st = ebbkc_count(g, k, &lo, stream);
    if (st == EBBKC_OK) {
        out_count[0] = lo;
        out_count[1] = 0;
        return EBBKC_OK;
    }
    if (st != EBBKC_E_OVERFLOW || g->last_total_ovf) return st;
    out_count[0] = g->last_total[0];
    out_count[1] = g->last_total[1];
    return EBBKC_OK;
}

ebbkc_status ebbkc_max_clique_size(ebbkc_graph* g, int32_t* out, void* stream) {
    if (!g || !out) return EBBKC_E_INVALID_ARG;
    if (g->n == 0) { *out = 0; return EBBKC_OK; }
    if (g->m == 0) { *out = 1; return EBBKC_OK; }
    // N_k > 0 is monotone in k (a k-clique holds (k-1)-cliques); N_2 = m > 0 and
    // N_k = 0 past tau + 2 (every k-clique lies in the sub-branch of its seed,
    // which has at most tau vertices)
    int lo = 2, hi = g->tau + 2;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        uint64_t c[2] = {0, 0};
        ebbkc_status st = ebbkc_count128(g, mid, c, stream);
        const bool some = st == EBBKC_OK ? (c[0] | c[1]) != 0 : st == EBBKC_E_OVERFLOW;
        if (st != EBBKC_OK && st != EBBKC_E_OVERFLOW) return st;
        if (some) lo = mid;
        else hi = mid - 1;
    }
    *out = lo;
    return EBBKC_OK;
}

ebbkc_status ebbkc_count_range(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, uint64_t* out_count,
                               void* stream) {
    if (!g || !out_count) return EBBKC_E_INVALID_ARG;
    if (k < 3) return EBBKC_E_K_RANGE;
    if (r_end < 0 || r_end > g->m) r_end = g->m;
    if (r_begin < 0 || r_begin > r_end) return EBBKC_E_INVALID_ARG;
    if (k - 2 > g->tau || r_begin == r_end) { *out_count = 0; return EBBKC_OK; }
    return ebb::count_impl(g, k, r_begin, r_end, nullptr, 0, nullptr, out_count, (hipStream_t)stream);
}

ebbkc_status ebbkc_count_seeds(ebbkc_graph* g, int32_t k, const int64_t* eids, int64_t ne, int32_t ptr_kind,
                               uint64_t* out, void* stream) {
    if (!g || (ne > 0 && (!eids || !out)) || ne < 0) return EBBKC_E_INVALID_ARG;
    return ebb::count_seeds_impl(g, k, eids, ne, ptr_kind, out, (hipStream_t)stream);
}

ebbkc_status ebbkc_list(ebbkc_graph* g, int32_t k, int64_t r_begin, int64_t r_end, int32_t* d_buf, uint64_t cap,
                        uint32_t flags, uint64_t* out_written, uint64_t* out_checksums, void* stream) {
    if (!g || !out_written || (cap > 0 && !d_buf)) return EBBKC_E_INVALID_ARG;
    uint64_t written = 0;
    ebbkc_status st = ebb::list_impl(g, k, r_begin, r_end, d_buf, cap, flags, &written, out_checksums,
                                     (hipStream_t)stream);
    if (st == EBBKC_OK || st == EBBKC_E_BUFFER_TOO_SMALL) *out_written = written;
    return st;
}

ebbkc_status ebbkc_export(const ebbkc_graph* gc, int32_t which, int32_t* dst, int32_t ptr_kind, void* stream) {
    ebbkc_graph* g = const_cast<ebbkc_graph*>(gc);
    if (!g || !dst) return EBBKC_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int32_t* src = nullptr;
    switch (which) {
        case EBBKC_ARR_SUPPORT: src = g->sup0; break;
        case EBBKC_ARR_RANK: src = g->rank; break;
        case EBBKC_ARR_LEVEL: src = g->level; break;
        case EBBKC_ARR_SUBSIZE: {
            ebbkc_status st = ebb::subsize_impl(g, s);
            if (st) return st;
            src = g->subsize;
            break;
        }
        case EBBKC_ARR_VERTEX_POS: src = g->vpos; break;
        case EBBKC_ARR_VERTEX_COLOR: src = g->vcol; break;
        default: return EBBKC_E_INVALID_ARG;
    }
    const bool per_vertex = which == EBBKC_ARR_VERTEX_POS || which == EBBKC_ARR_VERTEX_COLOR;
    const int64_t len = per_vertex ? (int64_t)g->n : g->m;
    if (len == 0) return EBBKC_OK;
    if (!src) return EBBKC_E_INVALID_ARG;  // not held under this handle's ordering
    hipMemcpyKind kind = ptr_kind == EBBKC_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (hipMemcpyAsync(dst, src, sizeof(int32_t) * (size_t)len, kind, s) != hipSuccess) return EBBKC_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return EBBKC_E_HIP;
    return EBBKC_OK;
}

ebbkc_status ebbkc_info_get(const ebbkc_graph* g, ebbkc_info* out) {
    if (!g || !out) return EBBKC_E_INVALID_ARG;
    out->n = g->n;
    out->m = g->m;
    out->tau = g->tau;
    out->rounds = g->rounds;
    out->max_degree = g->max_degree;
    out->device_bytes = g->device_bytes;
    out->prepare_ms = g->prepare_ms;
    return EBBKC_OK;
}

ebbkc_status ebbkc_last_timing(const ebbkc_graph* g, double out_ms[4]) {
    if (!g || !out_ms) return EBBKC_E_INVALID_ARG;
    for (int i = 0; i < 4; ++i) out_ms[i] = g->last_ms[i];
    return EBBKC_OK;
}

ebbkc_status ebbkc_last_work(const ebbkc_graph* g, uint64_t out[4]) {
    if (!g || !out) return EBBKC_E_INVALID_ARG;
    for (int i = 0; i < 4; ++i) out[i] = g->last_work[i];
    return EBBKC_OK;
}

ebbkc_status ebbkc_last_work_class(const ebbkc_graph* g, int32_t width_class, uint64_t out[4]) {
    if (!g || !out || width_class < 1 || width_class > 4) return EBBKC_E_INVALID_ARG;
    for (int i = 0; i < 4; ++i) out[i] = g->last_work_class[width_class - 1][i];
    return EBBKC_OK;
}

}  // extern "C"
