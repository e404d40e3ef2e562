// search.hip -- the EBBkC-C_Rec search over arena sub-branches (one
// wavefront per task).
//
// A task is a seed's g_i (from the arena, or built in LDS by the task) and a
// range [x0, x1) of first vertices of the root's children; light seeds are
// one task, heavy seeds one task per range of root vertices.  While some
// waves wait for work, a node can also be handed to one of them through a
// device queue.  On the DAG of g_i (vertices in colour order, edges
// low -> high) a node (P, l):
//   * is pruned when |P| < l (Algorithm EBBkC);
//   * at l = 1 counts |P|, at l = 2 the edges inside P;
//   * at l >= 3 is finished in closed form when P is a clique, C(|P|, l), or
//     a 2-plex, sum_j C(p, j) 2^j C(f, l-j) with f full vertices and p
//     non-adjacent pairs (Section 5, Algorithm kC2Plex);
//   * at l = 3 counts the triangles inside P;
//   * otherwise branches on every DAG edge x->y inside P into
//     P' = P & N+(x) & N+(y), l-2, skipping children by Rule (1)
//     (col x < l or col y < l-1) and Rule (2) (fewer than l-2 colours in P')
//     (Section 4.3, Algorithm EBBkC-C).
// Nodes with l = 4 or 5 hand their children (l = 2 or 3) to lanes, one child
// per lane, after renumbering onto one word fewer when the node's candidate
// set fits; everything above is wave-uniform with the lanes owning rows.
#include <type_traits>

#include "arena.h"
#include "build.h"
#include "device_util.h"

namespace ebb {

// C(n, r) for n < BIN_N, r < BIN_R, saturated to UINT64_MAX when it does not fit
constexpr int BIN_N = 1025, BIN_R = 65;
__device__ uint64_t g_binom[BIN_N * BIN_R];

__global__ void k_binom_init() {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= BIN_N) return;
    unsigned __int128 c = 1;
    bool sat = false;
    g_binom[n * BIN_R + 0] = 1;
    for (int r = 1; r < BIN_R; ++r) {
        if (r > n) { g_binom[n * BIN_R + r] = 0; continue; }
        if (!sat) {
            c = c * (unsigned __int128)(n - r + 1) / (unsigned __int128)r;
            if (c > (unsigned __int128)UINT64_MAX) sat = true;
        }
        g_binom[n * BIN_R + r] = sat ? UINT64_MAX : (uint64_t)c;
    }
}

namespace {

// C(n, r) or UINT64_MAX if it does not fit 64 bits
__device__ uint64_t binom(int n, int r) {
    if (r < 0 || r > n) return 0;
    if (r > n - r) r = n - r;
    if (n < BIN_N && r < BIN_R) return g_binom[n * BIN_R + r];
    unsigned __int128 c = 1;
    for (int j = 1; j <= r; ++j) {
        c = c * (unsigned __int128)(n - r + j) / (unsigned __int128)j;
        if (c > (unsigned __int128)UINT64_MAX) return UINT64_MAX;
    }
    return (uint64_t)c;
}

typedef unsigned __int128 u128;
constexpr u128 U128_MAX = ~(u128)0;

// C(n, r) for n <= 257, r <= 128 in 128 bits (Pascal's rule, built once per
// device); both words all ones when it does not fit
constexpr int B128_N = 258, B128_R = 129;
__device__ uint64_t g_binom128[B128_N * B128_R * 2];

__global__ void k_binom128_init() {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int n = 0; n < B128_N; ++n) {
        for (int r = 0; r < B128_R; ++r) {
            u128 v;
            bool sat = false;
            if (r == 0) v = 1;
            else if (r > n) v = 0;
            else {
                const uint64_t* a = &g_binom128[((n - 1) * B128_R + r - 1) * 2];
                const uint64_t* b = &g_binom128[((n - 1) * B128_R + r) * 2];
                const bool sa = a[0] == ~0ull && a[1] == ~0ull, sb = b[0] == ~0ull && b[1] == ~0ull;
                const u128 x = ((u128)a[1] << 64) | a[0], y = ((u128)b[1] << 64) | b[0];
                v = x + y;
                sat = sa || sb || v < x;
            }
            uint64_t* o = &g_binom128[(n * B128_R + r) * 2];
            o[0] = sat ? ~0ull : (uint64_t)v;
            o[1] = sat ? ~0ull : (uint64_t)(v >> 64);
        }
    }
}

// C(n, r) exactly in 128 bits; sets ovf when it does not fit
__device__ __forceinline__ u128 binom128(int n, int r, bool& ovf) {
    if (r < 0 || r > n) return 0;
    if (r > n - r) r = n - r;
    if (r == 0) return 1;
    if (n >= B128_N) { ovf = true; return 0; }
    const uint64_t* e = &g_binom128[(n * B128_R + r) * 2];
    const uint64_t lo = e[0], hi = e[1];
    if (lo == ~0ull && hi == ~0ull) { ovf = true; return 0; }
    return ((u128)hi << 64) | lo;
}

// a * b in 128 bits; sets ovf when it does not fit
__device__ __forceinline__ u128 mul128(u128 a, u128 b, bool& ovf) {
    const uint64_t ah = (uint64_t)(a >> 64), al = (uint64_t)a, bh = (uint64_t)(b >> 64), bl = (uint64_t)b;
    if (ah && bh) { ovf = true; return 0; }
    const u128 low = (u128)al * bl;
    const u128 mid = (u128)ah * bl + (u128)al * bh;  // one of the two terms is zero
    if (mid >> 64) { ovf = true; return 0; }
    const u128 r = low + (mid << 64);
    if (r < low) { ovf = true; return 0; }
    return r;
}

// l-cliques of a 2-plex with f vertices adjacent to all others and p
// non-adjacent pairs: sum_j C(p,j) 2^j C(f, l-j), exactly in 128 bits
__device__ u128 twoplex_count(int f, int p, int l, bool& ovf) {
    u128 s = 0;
    const int jmax = p < l ? p : l;
    for (int j = 0; j <= jmax; ++j) {
        if (l - j > f) continue;
        u128 t = mul128(binom128(p, j, ovf), binom128(f, l - j, ovf), ovf);
        if (t == 0) continue;
        if (j >= 128 || (t >> (127 - j)) != 0) { ovf = true; return 0; }
        t <<= j;
        s += t;
        if (s < t) { ovf = true; return 0; }
    }
    return s;
}

// exact 128-bit accumulator with an overflow flag
struct Acc {
    u128 v;
    bool ovf;
    __device__ void add(u128 x) {
        v += x;
        ovf |= v < x;
    }
    __device__ uint64_t lo() const { return (uint64_t)v; }
    __device__ uint64_t hi() const { return (uint64_t)(v >> 64); }
};

template <int W>
struct Frame {
    uint64_t P[W];
    uint64_t R[W];
    int32_t x, l, y, pad;
};

// children queued per node before the lanes count them (room for one more x)
constexpr int QRUN = 256, QCAP = QRUN + 256;

template <int W>
struct SearchMem {
    uint64_t rows[64 * W][W];
    int16_t col[64 * W];
    int16_t md[64 * W];      // missing pairs per vertex inside the set being counted
    int16_t vl[64 * W];      // that set's vertices in order, one per lane
    int32_t pq[2][QCAP];     // queued children |Q| << 16 | x << 8 | y (and a sort buffer)
    Frame<W> fr[LDS_FRAMES];
    // a node's candidate set renumbered onto W - 1 words (compact_set, W = 2
    // and 3): rows of up to 64 (W - 1) vertices, and their colours
    uint64_t crow[W == 2 || W == 3 ? 64 * (W - 1) * (W - 1) : 1];
    int16_t ccol[W == 2 || W == 3 ? 64 * (W - 1) : 1];
};

// nodes with fewer candidates are not renumbered onto narrower rows
constexpr int COMPACT_MIN = 16;

// The p vertices of P (p <= 64 WV, WV < W) renumbered 0 .. p-1 in ascending
// order, with their rows restricted to P and renumbered likewise (WV words)
// and their colours.  The order is kept, so the DAG (lower index first), the
// colour order and every clique inside P are the same; the node's leaves
// then run on WV-word rows.
template <int W, int WV>
__device__ void compact_set(const SearchMem<W>& M, const uint64_t (&P)[W], uint64_t (*rows_out)[WV],
                            int16_t* col_out) {
    const int lane = lane_id();
    int base = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        if (!P[q]) continue;
        if ((P[q] >> lane) & 1) {
            const int v = 64 * q + lane;
            const int idx = base + popc64(P[q] & lanemask_lt());
            uint64_t nr[WV];
#pragma unroll
            for (int z = 0; z < WV; ++z) nr[z] = 0;
            uint64_t cur = 0;
            int t = 0;
#pragma unroll
            for (int qq = 0; qq < W; ++qq) {
                const uint64_t rw = M.rows[v][qq];
                uint64_t bq = P[qq];
                while (bq) {
                    const int b = __builtin_ctzll(bq);
                    bq &= bq - 1;
                    cur |= ((rw >> b) & 1ull) << (t & 63);
                    if ((t & 63) == 63) {
#pragma unroll
                        for (int z = 0; z < WV; ++z)
                            if (z == (t >> 6)) nr[z] = cur;
                        cur = 0;
                    }
                    ++t;
                }
            }
            if (t & 63) {
#pragma unroll
                for (int z = 0; z < WV; ++z)
                    if (z == (t >> 6)) nr[z] = cur;
            }
#pragma unroll
            for (int z = 0; z < WV; ++z) rows_out[idx][z] = nr[z];
            col_out[idx] = M.col[v];
        }
        base += popc64(P[q]);
    }
    wave_sync();
}

// ---------------------------------------------------------------- per-lane leaves
// One lane counts the cliques of one child candidate set Q from LDS rows.

template <int W>
__device__ __forceinline__ uint64_t lane_edges(const uint64_t (*rows)[W], const uint64_t (&Q)[W]) {
    uint32_t e2 = 0;
#pragma unroll
    for (int wz = 0; wz < W; ++wz) {
        uint64_t bits = Q[wz];
        while (bits) {
            const int z = wz * 64 + __builtin_ctzll(bits);
            bits &= bits - 1;
#pragma unroll
            for (int w = 0; w < W; ++w) e2 += popc64(Q[w] & rows[z][w]);
        }
    }
    return e2 / 2;
}

// Triangles inside Q.  Dense Q (missing pairs M <= edges E): T = C(q,3) -
// M(q-2) + sum_v C(m_v,2) - T_c with m_v the missing pairs at v and T_c the
// triangles of missing pairs; sparse Q: common out-neighbours along the DAG
// edges.  dense_hint (the parent set is dense, so Q almost surely is) takes
// the degrees and T_c in one pass over Q with 32-bit bit iteration, and falls
// back to the sparse pass if Q turns out sparse after all; otherwise the
// degrees come first and only the needed pass follows.
template <int W>
__device__ __forceinline__ uint64_t lane_triangles(const uint64_t (*rows)[W], const uint64_t (&Q)[W], bool dense_hint,
                                                   uint64_t& ops) {
    constexpr int H = 2 * W;  // 32-bit halves of a row
    const int q = popcW(Q);
    if (q < 3) return 0;
    const uint64_t q64 = (uint64_t)q;
    const uint64_t C3 = q64 * (q64 - 1) * (q64 - 2) / 6;
    uint32_t e2 = 0, s2 = 0, t = 0;
    if (dense_hint) {
        uint32_t Qh[H];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            Qh[2 * w] = (uint32_t)Q[w];
            Qh[2 * w + 1] = (uint32_t)(Q[w] >> 32);
        }
#pragma unroll
        for (int hz = 0; hz < H; ++hz) {
            uint32_t bits = Qh[hz];
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1;
                const uint32_t* rz = reinterpret_cast<const uint32_t*>(rows[32 * hz + b]);
                uint32_t Cz[H];  // missing pairs z-y inside Q with y > z
                int d = 0;
#pragma unroll
                for (int g = 0; g < H; ++g) {
                    const uint32_t row = rz[g];
                    d += __builtin_popcount(Qh[g] & row);
                    if (g > hz) Cz[g] = Qh[g] & ~row;
                    else if (g == hz) Cz[g] = Qh[g] & ~row & (b == 31 ? 0u : (~0u << (b + 1)));
                    else Cz[g] = 0;
                }
                e2 += d;
                const int cm = q - 1 - d;
                s2 += (uint32_t)(cm * (cm - 1) / 2);
#pragma unroll
                for (int gy = hz; gy < H; ++gy) {
                    while (Cz[gy]) {
                        const uint32_t* ry = reinterpret_cast<const uint32_t*>(rows[32 * gy + __builtin_ctz(Cz[gy])]);
                        Cz[gy] &= Cz[gy] - 1;
#pragma unroll
                        for (int g = gy; g < H; ++g) t += __builtin_popcount(Cz[g] & ~ry[g]);
                    }
                }
            }
        }
        const uint64_t Mp = (q64 * (q64 - 1) - e2) / 2, E = e2 / 2;
        ops += (uint64_t)q * W;
        if (Mp == 0) return C3;
        if (Mp <= E) {
            ops += Mp * W;
            return C3 - Mp * (q64 - 2) + s2 - t;
        }
        t = 0;  // sparse after all: the pass along edges below
    } else {
#pragma unroll
        for (int wz = 0; wz < W; ++wz) {
            uint64_t bits = Q[wz];
            while (bits) {
                const int z = wz * 64 + __builtin_ctzll(bits);
                bits &= bits - 1;
                int d = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) d += popc64(Q[w] & rows[z][w]);
                e2 += d;
                const int cm = q - 1 - d;
                s2 += (uint32_t)(cm * (cm - 1) / 2);
            }
        }
        ops += (uint64_t)q * W;
    }
    const uint64_t Mp = (q64 * (q64 - 1) - e2) / 2, E = e2 / 2;
    if (Mp == 0) return C3;
    const bool dense = Mp <= E;
    ops += (dense ? Mp : E) * W;
#pragma unroll
    for (int wz = 0; wz < W; ++wz) {
        uint64_t bits = Q[wz];
        while (bits) {
            const int z = wz * 64 + __builtin_ctzll(bits);
            bits &= bits - 1;
            uint64_t Cz[W];  // missing (dense) or present (sparse) pairs z-y, y > z, inside Q
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t row = dense ? ~rows[z][w] : rows[z][w];
                Cz[w] = Q[w] & row & upper_mask(z, w);
            }
#pragma unroll
            for (int wy = 0; wy < W; ++wy) {
                while (Cz[wy]) {
                    const int y = wy * 64 + __builtin_ctzll(Cz[wy]);
                    Cz[wy] &= Cz[wy] - 1;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const uint64_t row = dense ? ~rows[y][w] : rows[y][w];
                        if (w >= wy) t += popc64(Cz[w] & row);
                    }
                }
            }
        }
    }
    return dense ? C3 - Mp * (q64 - 2) + s2 - t : (uint64_t)t;
}

// l-cliques of a 3-plex P (every vertex misses at most two others of P):
// the coefficient of x^l in the independence polynomial of the missing
// pairs H[P], a disjoint union of paths and cycles; Algorithm kCtPlex
// reaches the same sets by branching on H.  Lanes walk the components from
// their vertices into length histograms; the product of path polynomials
// (sum_i C(L-i+1, i) x^i) and cycle polynomials (sum_i [C(L-i, i) +
// C(L-i-1, i-1)] x^i) is formed in LDS, lane j mod 64 owning coefficient j.
// Needs l < pc (so l < 256); sets ovf when the coefficient reaches 2^128.
template <int W>
__device__ __forceinline__ u128 threeplex_count(SearchMem<W>& M, const uint64_t (&P)[W], int pc, int l, bool& ovf) {
const int lane = lane_id();
        int32_t* hp = M.pq[0];   // paths by length
        int32_t* hcy = M.pq[1];  // cycles by length
        for (int i = lane; i < 257; i += 64) { hp[i] = 0; hcy[i] = 0; }
        {
            int base = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                if ((P[q] >> lane) & 1) M.vl[base + popc64(P[q] & lanemask_lt())] = (int16_t)(lane + 64 * q);
                base += popc64(P[q]);
            }
        }
        wave_sync();
        const int rounds = (pc + 63) >> 6;
        for (int t = 0; t < rounds; ++t) {
            const int j = 64 * t + lane;
            if (j < pc) {
                const int v = M.vl[j];
                int mv = -1;  // P & ~row(v) holds v itself
#pragma unroll
                for (int w = 0; w < W; ++w) mv += popc64(P[w] & ~M.rows[v][w]);
                M.md[v] = (int16_t)mv;
            }
        }
        wave_sync();
        // an H-neighbour of cur other than avoid (-1: none)
        auto hnext = [&](int cur, int avoid) -> int {
            int r = -1;
#pragma unroll
            for (int w = W - 1; w >= 0; --w) {
                uint64_t h = P[w] & ~M.rows[cur][w];
                if (w == (cur >> 6)) h &= ~(1ull << (cur & 63));
                if (avoid >= 0 && w == (avoid >> 6)) h &= ~(1ull << (avoid & 63));
                if (h) r = w * 64 + __builtin_ctzll(h);
            }
            return r;
        };
        for (int t = 0; t < rounds; ++t) {
            const int j = 64 * t + lane;
            if (j >= pc) continue;
            const int v = M.vl[j];
            const int mv = M.md[v];
            if (mv <= 1) {  // end of a path (or a lone vertex): walk to the other end
                int prev = -1, cur = v, L = 1;
                if (mv == 1) {
                    for (;;) {
                        const int nx = hnext(cur, prev);
                        prev = cur;
                        cur = nx;
                        ++L;
                        if (M.md[cur] <= 1) break;
                    }
                }
                if (mv == 0 || v < cur) atomicAdd(&hp[L], 1);
            } else {  // on a cycle if the walk comes back to v without meeting an end
                int prev = v, cur = hnext(v, -1), L = 1, mn = v;
                bool cyc = true;
                while (cur != v) {
                    if (M.md[cur] <= 1) { cyc = false; break; }
                    mn = cur < mn ? cur : mn;
                    const int nx = hnext(cur, prev);
                    prev = cur;
                    cur = nx;
                    ++L;
                }
                if (cyc && mn == v) atomicAdd(&hcy[L], 1);
            }
        }
        wave_sync();
        // the histograms move to md / vl (component length L at index L - 1,
        // L <= pc <= 64 W) so that pq can hold the product's coefficients
        for (int L = 1 + lane; L <= pc; L += 64) {
            M.md[L - 1] = (int16_t)hp[L];
            M.vl[L - 1] = (int16_t)hcy[L];
        }
        wave_sync();
        // coefficient j = lane + 64 q of the running product lives at poly[j]
        // (degrees 0..l, l <= 255); a coefficient that reached 2^128 is
        // flagged in the wave-uniform bit set fl and stays flagged, since
        // every factor has positive coefficients up to its degree
        u128* poly = reinterpret_cast<u128*>(&M.pq[0][0]);
        const int Q = (l >> 6) + 1;
#pragma unroll
        for (int q = 0; q < W; ++q)
            if (q < Q) poly[lane + 64 * q] = (lane + 64 * q == 0) ? (u128)1 : (u128)0;
        uint64_t fl[W];
#pragma unroll
        for (int q = 0; q < W; ++q) fl[q] = 0;
        wave_sync();
        auto flagged = [&](int j) -> bool {
            bool f = false;
#pragma unroll
            for (int q = 0; q < W; ++q)
                if ((j >> 6) == q) f = (fl[q] >> (j & 63)) & 1;
            return f;
        };
        // poly <- poly * sum_{i <= deg} coef(i) x^i, truncated at degree l
        auto mulpoly = [&](int deg, auto coef) {
            u128 nr[W];
            bool no[W];
#pragma unroll
            for (int q = 0; q < W; ++q) { nr[q] = 0; no[q] = false; }
            const int imax = deg < l ? deg : l;
            for (int i = 0; i <= imax; ++i) {
                bool co = false;
                const u128 c = coef(i, co);
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const int j = lane + 64 * q;
                    if (q >= Q || j > l || j < i || no[q]) continue;
                    if (flagged(j - i)) { no[q] = true; continue; }
                    const u128 o = poly[j - i];
                    if (!o) continue;
                    if (co) { no[q] = true; continue; }
                    bool mo = false;
                    const u128 t = mul128(c, o, mo);
                    nr[q] += t;
                    no[q] = mo || nr[q] < t;
                }
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < W; ++q) {
                if (q < Q) poly[lane + 64 * q] = nr[q];
                fl[q] |= uni64(__ballot(no[q]));
            }
            wave_sync();
        };
        for (int L = 1; L <= pc; ++L) {
            const int np = M.md[L - 1], nc = M.vl[L - 1];
            if (np && L == 1) {
                mulpoly(np, [&](int i, bool& o) { return binom128(np, i, o); });
            } else if (np && L == 2) {
                mulpoly(np, [&](int i, bool& o) {
                    if (i >= 128) { o = true; return (u128)0; }
                    return mul128(binom128(np, i, o), (u128)1 << i, o);
                });
            } else {
                for (int rep = 0; rep < np; ++rep)
                    mulpoly((L + 1) / 2, [&](int i, bool& o) { return binom128(L - i + 1, i, o); });
            }
            for (int rep = 0; rep < nc; ++rep)
                mulpoly(L / 2, [&](int i, bool& o) {
                    if (i == 0) return (u128)1;
                    const u128 x = binom128(L - i, i, o), y = binom128(L - i - 1, i - 1, o);
                    if (x + y < x) o = true;
                    return x + y;
                });
        }
        ovf |= flagged(l);
        const u128 res = poly[l];
        wave_sync();
        return res;
}

// l-cliques of a t-plex P (every vertex misses at most t-1 others of P),
// any t, by Algorithm kCtPlex: the vertices adjacent to all others (I, the
// isolated vertices of the inverse graph) are taken in closed form -- a node
// (S', C, l') contributes the C(|I|, l') ways to finish S' from I -- and the
// branching runs on the rest: the child of v_i in C (in order) keeps the
// vertices of C after v_i that are adjacent to v_i (Eq. kCtPlex: C minus v_1..
// v_i minus v_i's neighbours in the inverse graph), l' - 1, when it still
// holds enough vertices with I.  Children with l' - 1 <= 1 are counted at
// once (l' - 1 = 1: |I| + |C_i|; 0: one clique).  Frames (C, l', last v)
// live in the child-queue area of LDS: depth <= l <= KCT_MAX_L.
constexpr int KCT_MAX_L = 96;

template <int W>
struct KctFrame {
    uint64_t C[W];
    int32_t l, cur;
};
static_assert(sizeof(KctFrame<4>) * KCT_MAX_L <= 2 * QCAP * sizeof(int32_t), "kCtPlex frames must fit the queue area");

template <int W>
__device__ u128 tplex_branch_count(SearchMem<W>& M, const uint64_t (&P)[W], int pc, int l, bool& ovf,
                                   uint64_t& nodes) {
    const int lane = lane_id();
    // I: vertices of P adjacent to all others of P
    uint64_t I[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        bool full = false;
        if ((P[q] >> lane) & 1) {
            int d = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) d += popc64(P[w] & M.rows[lane + 64 * q][w]);
            full = d == pc - 1;
        }
        I[q] = uni64(ballot(full));
    }
    const int nI = popcW(I);
    auto add = [&](u128& acc, u128 x) {
        acc += x;
        ovf |= acc < x;
    };
    KctFrame<W>* fr = reinterpret_cast<KctFrame<W>*>(&M.pq[0][0]);
    u128 total = 0;
    add(total, binom128(nI, l, ovf));  // the root: all l vertices from I
    int sp = 0;
    if (lane == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) fr[0].C[w] = P[w] & ~I[w];
        fr[0].l = l;
        fr[0].cur = -1;
    }
    wave_sync();
    while (sp >= 0) {
        uint64_t C[W];
#pragma unroll
        for (int w = 0; w < W; ++w) C[w] = uni64(fr[sp].C[w]);
        const int lf = uniform_i32(fr[sp].l), cur = uniform_i32(fr[sp].cur);
        int v = -1;  // next vertex of C after cur
#pragma unroll
        for (int w = W - 1; w >= 0; --w) {
            const uint64_t b = C[w] & (cur < 0 ? ~0ull : upper_mask(cur, w));
            if (b) v = 64 * w + __builtin_ctzll(b);
        }
        if (v < 0) {
            --sp;
            continue;
        }
        if (lane == 0) fr[sp].cur = v;
        const int lc = lf - 1;
        ++nodes;
        if (lc == 0) {
            add(total, 1);
            wave_sync();
            continue;
        }
        uint64_t Ci[W];
#pragma unroll
        for (int w = 0; w < W; ++w) Ci[w] = C[w] & M.rows[v][w] & upper_mask(v, w);
        const int ci = popcW(Ci);
        if (ci + nI < lc) {
            wave_sync();
            continue;
        }
        if (lc == 1) {  // C(|I|, 1) from I, and each vertex of C_i
            add(total, (u128)(nI + ci));
            wave_sync();
            continue;
        }
        add(total, binom128(nI, lc, ovf));  // the child: the rest from I
        if (lane == 0) {
#pragma unroll
            for (int w = 0; w < W; ++w) fr[sp + 1].C[w] = Ci[w];
            fr[sp + 1].l = lc;
            fr[sp + 1].cur = -1;
        }
        ++sp;
        wave_sync();
    }
    wave_sync();
    return total;
}

}  // namespace

// The build's work areas alias the search's per-vertex scratch, child queue
// and LDS frames (md .. fr), which the search writes before it reads.
template <int W>
constexpr bool build_fits() {
    return build_scratch_bytes<W>() <= (int)(sizeof(SearchMem<W>) - offsetof(SearchMem<W>, md));
}
static_assert(build_fits<1>() && build_fits<2>() && build_fits<3>() && build_fits<4>(),
              "sub-branch build scratch must fit the search's LDS");

// ---------------------------------------------------------------- split queue
// Counters are touched once per queue operation, sequentially consistent at
// device scope, so that a wave that sees no working wave also sees every item
// pushed before the last one stopped.
__device__ __forceinline__ unsigned long long sq_load(unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long sq_add(unsigned long long* p, long long v) {
    return __hip_atomic_fetch_add(p, (unsigned long long)v, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
}
// a hint only (whether to push): no ordering, no wait for the wave's other
// memory operations
__device__ __forceinline__ unsigned long long sq_peek(unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
constexpr int SQ_POLL_BUSY = 256, SQ_POLL_HUNGRY = 4;
constexpr uint64_t SQ_POLL_TICKS = 2000;  // 20 us of the 100 MHz clock
// longest time a wave waits while the queue shows no progress (no item
// claimed or reserved, no change in the working waves) before it gives up
// with ERR_QUEUE (constant-rate clock of 100 MHz: 60 s); also at most
// SQ_WAIT_SPINS sleeps (each at least 64 * 32 clocks), so the wait ends even
// if that clock did not advance
constexpr uint64_t SQ_WAIT_TICKS = 6000000000ull;
constexpr uint64_t SQ_WAIT_SPINS = 1ull << 26;

// An idle wave claims a queued node: returns its index once its producer has
// written it, or -1 when no wave is working and the queue is empty (then no
// item can appear any more: an item is pushed only by a working wave, before
// that wave stops counting as working) or after SQ_WAIT_TICKS without work
// (ERR_QUEUE).  A claim takes the head first and counts the wave as working
// after it; a wave in between may process that node while others have
// finished, and handles whatever it pushes itself.  Idle polling backs off
// and reads the counters without ordering (an ordered atomic would also
// drop the compute unit's vector cache, which the working waves beside it
// use for their spilled registers); only a claim and the final check that
// nothing is left are ordered.
__device__ int64_t queue_take(const SearchArgs& a) {
    unsigned long long* sq = a.sq;
    uint64_t t0 = wall_clock64();
    unsigned long long seen_h = ~0ull, seen_r = ~0ull, seen_b = ~0ull;
    int nap = 1;
    for (uint64_t spin = 0;; ++spin) {
        long long got = -1;
        int done = 0;
        if (lane_id() == 0) {
            const unsigned long long h = sq_peek(&sq[SQ_HEAD]), r = sq_peek(&sq[SQ_RESERVE]);
            const unsigned long long bz = sq_peek(&sq[SQ_BUSY]);
            if (h != seen_h || r != seen_r || bz != seen_b) {  // progress: the wait starts again
                seen_h = h;
                seen_r = r;
                seen_b = bz;
                t0 = wall_clock64();
                spin = 0;
            }
            if (h < r && atomicCAS(&sq[SQ_HEAD], h, h + 1) == h) {
                got = (long long)h;
                sq_add(&sq[SQ_BUSY], 1);
                sq_add(&sq[SQ_IDLE], -1);
            } else if (h >= r && bz == 0 && sq_load(&sq[SQ_BUSY]) == 0 &&
                       sq_load(&sq[SQ_HEAD]) >= sq_load(&sq[SQ_RESERVE])) {
                done = 1;
            } else if (wall_clock64() - t0 > SQ_WAIT_TICKS || spin > SQ_WAIT_SPINS) {
                atomicOr(a.err, ERR_QUEUE);
                done = 1;
            }
            if (got >= 0) {  // the producer reserved the slot before writing it
                for (uint64_t wspin = 0;
                     __hip_atomic_load(&a.squeue[got].ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0; ++wspin) {
                    if (wall_clock64() - t0 > SQ_WAIT_TICKS || wspin > SQ_WAIT_SPINS) {
                        atomicOr(a.err, ERR_QUEUE);
                        got = -1;
                        done = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
        }
        got = (long long)uni64((uint64_t)__shfl(got, 0, 64));
        done = uniform_i32(__shfl(done, 0, 64));
        if (got >= 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every lane sees the item
            return got;
        }
        if (done) return -1;
        for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(64);
        nap = nap < 32 ? 2 * nap : 32;
    }
}

// BUILD = false: each task's g_i is loaded from the arena.  BUILD = true
// (batches too large for arenas): the task's slot is its seed edge id in
// graph task_graph[i], and the wave builds g_i in LDS first (build.h).
template <int W, bool BUILD>
__global__ __launch_bounds__(256, (W <= 2 ? 4 : (W <= 3 ? 3 : 2))) void k_search(SearchArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SearchMem<W>& M = reinterpret_cast<SearchMem<W>*>(smem_raw)[threadIdx.x / 64];
    Frame<W>* gfr = a.gframes ? reinterpret_cast<Frame<W>*>(a.gframes) +
                                    ((int64_t)blockIdx.x * 4 + threadIdx.x / 64) * GLOBAL_FRAMES
                              : nullptr;
    // frames past the LDS ones live in this wave's slab of device memory;
    // every lane writes them (identical values) and reads back its own stores
    auto FR = [&](int d) -> Frame<W>& { return d < LDS_FRAMES ? M.fr[d] : gfr[d - LDS_FRAMES]; };
    const int lane = lane_id();
    const int opts = a.opts;
    const bool rule1 = opts & OPT_RULE1, rule2 = opts & OPT_RULE2, et = opts & OPT_ET;
    const bool work = opts & OPT_WORK;
    Acc acc{0, false};
    uint64_t wk_tasks = 0, wk_nodes = 0, wk_ops = 0;
    const uint64_t t_wave0 = work ? wall_clock64() : 0;
    // runtime splitting: a wave counts as working from its start until the
    // static tasks run out, then takes queued nodes until none is left
    const bool splitting = a.squeue != nullptr;
    if (splitting && lane == 0) sq_add(&a.sq[SQ_BUSY], 1);
    bool on_queue = false, took_item = false;
    int poll_in = 0;      // candidate nodes until the queue counters are read again
    uint64_t poll_t = 0;  // when they were read last
    bool hungry = false;  // some wave waited for work at the last reading
    // lane j: the least |P| with C(|P|, j) >= split_bound (a node with l = j
    // and fewer candidates is never handed over), so that the test per node
    // is a lane read instead of a table load
    int push_pmin = 1 << 20;
    if (splitting) {
        const int j = lane;
        int lo = j > 0 ? j : 1, hi = 64 * MAX_W + 1;  // C(hi, j) may stay below the bound: then never
        if (j > 0 && binom(hi, j) >= a.split_bound) {
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (binom(mid, j) >= a.split_bound) hi = mid; else lo = mid + 1;
            }
            push_pmin = lo;
        }
    }

    for (;;) {
        unsigned long long it = 0;
        int64_t qitem = -1;
        if (!on_queue) {
            if (lane == 0) it = atomicAdd(a.next, 1ull);
            it = uni64(__shfl(it, 0, 64));
            if ((int64_t)it >= a.ntasks) {
                if (!splitting) break;
                on_queue = true;
                if (lane == 0) {
                    sq_add(&a.sq[SQ_IDLE], 1);
                    sq_add(&a.sq[SQ_BUSY], -1);
                }
            }
        }
        if (on_queue) {
            if (took_item && lane == 0) {  // the last queued node is done (its pushes are visible)
                sq_add(&a.sq[SQ_IDLE], 1);
                sq_add(&a.sq[SQ_BUSY], -1);
            }
            qitem = queue_take(a);
            if (qitem < 0) break;
            took_item = true;
            it = uni64((uint64_t)a.squeue[qitem].it);
        }
        const int64_t task = a.tasks[it];
        const int64_t slot = task_slot(task);
        // a queued node is a whole node below the root: every first vertex
        const int x0 = qitem >= 0 ? 0 : task_x0(task);
        const int x1 = qitem >= 0 ? 64 * W : task_x1(task);
        const int gi = a.task_graph ? uniform_i32(a.task_graph[it]) : 0;
        const int k = a.graph_k ? uniform_i32(a.graph_k[gi]) : a.k;
        int c = 0;
        int64_t ro = 0, vo = 0;
        if constexpr (BUILD) {
            c = uniform_i32(a.bviews[gi].subsize[slot]);
        } else {
            const ArenaView& A = a.views ? a.views[gi] : a.A;
            c = uniform_i32(A.seed_c[slot]);
            ro = A.row_off[slot];
            vo = A.vtx_off[slot];
        }
        // t of the closed forms: fixed, or 2 when 2k <= tau and 3 above (Section 6.1)
        const int tau_g = a.graph_tau ? uniform_i32(a.graph_tau[gi]) : a.tau;
        const int tpl = a.tplex > 0 ? a.tplex : (2 * k <= tau_g ? 2 : 3);
        const bool t2 = et && tpl >= 2, t3 = et && tpl >= 3, t4 = et && tpl >= 4;
        wk_tasks += work;
        Acc tacc{0, false};
        if (k == 3) {  // l = 1 at the root: |V(g_i)| triangles through the seed edge
            tacc.add((uint64_t)c);
            goto task_done;
        }

        if constexpr (BUILD) {
            // ---- build g_i in LDS, vertices in colour order (build.h)
            const BuildGraph& B = a.bviews[gi];
            const BuildScratch<W> S = BuildScratch<W>::carve(&M.md[0]);
            const int32_t e = (int32_t)slot;
            uint32_t twoE = 0;
            if (build_subbranch<W>(B.G, B.G.eu[e], B.G.ev[e], B.G.rank[e], c, B.vcol, M.rows, M.col, S, &twoE) < 0) {
                if (lane == 0) atomicOr(a.err, ERR_WIDTH);
                goto task_done;
            }
            int npos[W];
            order_positions<W>(c, M.col, S, npos);
            uint64_t nr[W][W];
            int16_t nc[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int i = lane + 64 * q;
                nc[q] = 0;
                if (i < c) {
                    relabelled_row<W>(M.rows, i, S, nr[q]);
                    nc[q] = M.col[i];
                }
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < W; ++q) {
                if (lane + 64 * q < c) {
#pragma unroll
                    for (int w = 0; w < W; ++w) M.rows[npos[q]][w] = nr[q][w];
                    M.col[npos[q]] = nc[q];
                }
            }
            wave_sync();
        } else {
            // ---- load the sub-branch into LDS (coalesced)
            const ArenaView& A = a.views ? a.views[gi] : a.A;
            for (int i = lane; i < c * W; i += 64) (&M.rows[0][0])[i] = A.rows[ro + i];
            for (int i = lane; i < c; i += 64) M.col[i] = A.col[vo + i];
            wave_sync();
        }
        {
        // colour class lane + 64 q (colour lane + 64 q + 1) occupies the
        // relabelled positions [cs0[q], cs1[q]) = [#(col > colour), #(col >= colour))
        int cs0[W], cs1[W];
        const int ncol = uniform_i32(M.col[0]);
        const int ncq = (ncol + 63) >> 6;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int cv = lane + 64 * q + 1;
            int lo = 0, hi = c;
            while (lo < hi) { int mid = (lo + hi) >> 1; if (M.col[mid] > cv) lo = mid + 1; else hi = mid; }
            const int s0 = lo;
            hi = c;
            while (lo < hi) { int mid = (lo + hi) >> 1; if (M.col[mid] >= cv) lo = mid + 1; else hi = mid; }
            cs0[q] = s0;
            cs1[q] = cv <= ncol ? lo : s0;
        }

        // Count a node that needs no branching: returns true and sets val, or
        // false when the node (l >= 4) must be branched on.
        auto finish = [&](const uint64_t (&P)[W], int l, u128& val) -> bool {
            const int pc = popcW(P);
            val = 0;
            if (work) { wk_nodes += 1; wk_ops += W; }
            if (pc < l) return true;
            if (l == 1) { val = (uint64_t)pc; return true; }
            int mn = 1 << 30, nf = 0;
            uint32_t dsum = 0, s2 = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                if ((P[q] >> lane) & 1) {
                    int d = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) d += popc64(P[w] & M.rows[lane + 64 * q][w]);
                    mn = d < mn ? d : mn;
                    nf += (d == pc - 1);
                    dsum += d;
                    const int cm = pc - 1 - d;
                    s2 += (uint32_t)(cm * (cm - 1) / 2);
                }
            }
            if (work) wk_ops += (uint64_t)pc * W;
            const uint64_t twoE = wsum_u32(dsum);
            if (l == 2) { val = twoE / 2; return true; }
            if (et) {
                const int mind = wmin_i32(mn);
                if (mind >= pc - 1) { val = binom128(pc, l, tacc.ovf); return true; }
                if (t2 && mind >= pc - 2) {
                    const int nfull = (int)wsum_u32((uint32_t)nf);
                    val = twoplex_count(nfull, (pc - nfull) / 2, l, tacc.ovf);
                    return true;
                }
                if (l == pc) { val = 0; return true; }  // P itself is not a clique
                if (t3 && mind >= pc - 3) {
                    val = threeplex_count<W>(M, P, pc, l, tacc.ovf);
                    return true;
                }
                if (t4 && mind >= pc - tpl && l <= KCT_MAX_L) {
                    uint64_t kn = 0;
                    val = tplex_branch_count<W>(M, P, pc, l, tacc.ovf, kn);
                    if (work) { wk_nodes += kn; wk_ops += kn * W; }
                    return true;
                }
            }
            if (l != 3) return false;
            // triangles inside P: dense -> missing-pair identity, sparse -> DAG edges
            const uint64_t p64 = (uint64_t)pc;
            const uint64_t Mp = (p64 * (p64 - 1) - twoE) / 2;
            uint32_t t = 0;
            const bool dense = Mp <= twoE / 2;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int z = lane + 64 * q;
                if ((P[q] >> lane) & 1) {
                    uint64_t Cz[W];
#pragma unroll
                    for (int w = 0; w < W; ++w)
                        Cz[w] = P[w] & (dense ? ~M.rows[z][w] : M.rows[z][w]) & upper_mask(z, w);
#pragma unroll
                    for (int wy = 0; wy < W; ++wy) {
                        while (Cz[wy]) {
                            const int y = wy * 64 + __builtin_ctzll(Cz[wy]);
                            Cz[wy] &= Cz[wy] - 1;
#pragma unroll
                            for (int w = 0; w < W; ++w) {
                                const uint64_t row = dense ? ~M.rows[y][w] : M.rows[y][w];
                                if (w >= wy) t += popc64(Cz[w] & row);
                            }
                        }
                    }
                }
            }
            if (work) wk_ops += (dense ? Mp : twoE / 2) * W;
            const uint64_t T = wsum_u32(t);
            if (dense) {
                const uint64_t S2 = wsum_u32(s2);
                val = p64 * (p64 - 1) * (p64 - 2) / 6 - Mp * (p64 - 2) + S2 - T;
            } else {
                val = T;
            }
            return true;
        };

        // 4-cliques inside R (r >= 4 vertices) from the missing pairs H of R:
        // inclusion-exclusion over the edge sets of H spanning at most four
        // vertices gives K4 = C(r,4) - M C(r-2,2) + P3 (r-3) + 2K2 - T (r-3)
        // - P4 - S3 + C4 + paw - diamond + K4(H), with P3 the 2-paths, 2K2
        // the disjoint pairs, T the triangles, P4 the 3-paths, S3 the 3-stars,
        // C4 the 4-cycles, paw, diamond and K4(H) the remaining 4-vertex
        // shapes of H.  All but C(r,4) + C(M,2) is a sum over the vertices,
        // missing pairs and 2-paths of H, taken by the lanes holding them
        // into S (12 times its value, so that every term is an integer).
        // Returns false, counting nothing, when H is too dense for this to
        // beat branching on the pairs of R.  (Spreading all pairs of R over
        // the lanes instead evens out vertices with many missing pairs, but
        // costs ~r^2 / 64 rounds even for a nearly complete R; on R-MAT s18
        // at k = 9 it made the search 1.7x slower.)
        auto k4_missing = [&](auto wv, const auto& R, auto rows, int r, bool whole, int64_t& S, uint64_t& uacc,
                              bool& rdense) -> bool {
            constexpr int WV = decltype(wv)::value;
            // the vertices of R, packed onto consecutive lanes
            {
                int base = 0;
#pragma unroll
                for (int q = 0; q < WV; ++q) {
                    if ((R[q] >> lane) & 1) M.vl[base + popc64(R[q] & lanemask_lt())] = (int16_t)(lane + 64 * q);
                    base += popc64(R[q]);
                }
            }
            wave_sync();
            const int rounds = (r + 63) >> 6;
            int msum = 0, cm2 = 0, lw = 0;
            for (int t = 0; t < rounds; ++t) {
                const int j = 64 * t + lane;
                if (j < r) {
                    const int v = M.vl[j];
                    int mv = -1;  // R & ~row(v) holds v itself
#pragma unroll
                    for (int w = 0; w < WV; ++w) mv += popc64(R[w] & ~rows[v][w]);
                    M.md[v] = (int16_t)mv;
                    msum += mv;
                    cm2 += mv * (mv - 1) / 2;
                    lw += mv + mv * (mv - 1) / 2;
                }
            }
            const int Msum = (int)wsum_u32((uint32_t)msum);
            const int64_t P3 = (int64_t)wsum_u32((uint32_t)cm2);
            // The lanes run in lockstep, so this evaluation takes as long as
            // its busiest lane (missing pairs + 2-paths at the vertices it
            // holds, ~15 instructions each) plus ~150 for the reductions.  The
            // alternative for one R = P & N+(x) of an l = 5 node is one child
            // y per lane counting the triangles of R & N+(y): ~35 instructions
            // per vertex of the largest child, ~ r * d, per 64 children (r of
            // them here, sharing rounds with the other x through the queue);
            // for a whole l = 4 node it is that for every x (~18 instructions
            // a step), ~ |E(R)| * d / 64 rounds of 64 children.
            const int lmax = wmax_i32(lw);
            const float pairs = 0.5f * (float)r * (float)(r - 1);
            const float E = pairs - 0.5f * (float)Msum, d = E / pairs;
            rdense = 2.0f * E >= pairs;
            const float cost = a.k4_weight * (15.0f * (float)lmax + 150.0f);
            const float alt = whole ? 18.0f * E * d * (float)r * d / 64.0f
                                    : 35.0f * (float)r * d * (float)r / 64.0f;
            if (!(a.k4_weight > 0.f) || cost > alt) return false;
            if (work) wk_ops += (uint64_t)(r + Msum + P3) * WV;
            const int64_t Mh = Msum / 2;
            const uint64_t r64 = (uint64_t)r;
            uacc += r64 * (r64 - 1) * (r64 - 2) * (r64 - 3) / 24 + (uint64_t)(Mh * (Mh - 1) / 2);
            if (Msum == 0) return true;
            wave_sync();  // md[] of every vertex of R
            const int64_t c2 = (int64_t)(r - 2) * (r - 3) / 2;
            for (int t = 0; t < rounds; ++t) {
                const int j = 64 * t + lane;
                if (j >= r) continue;
                const int v = M.vl[j];
                uint64_t hv[WV];
#pragma unroll
                for (int w = 0; w < WV; ++w)
                    hv[w] = R[w] & ~rows[v][w] & (w == (v >> 6) ? ~(1ull << (v & 63)) : ~0ull);
                const int64_t mv = M.md[v];
                if (mv == 0) continue;
                S += -6 * c2 * mv + 12 * (int64_t)(r - 4) * (mv * (mv - 1) / 2) - 2 * mv * (mv - 1) * (mv - 2);
                // missing pairs v-u: codegree cc in H (triangles, diamonds,
                // paws), the 3-paths through v-u, K4(H).  Per-v sums in 32 bits:
                // t2 = sum cc over all u; over u > v: a1 = sum cc, a2 = sum cc^2,
                // a3 = sum (m_u - 1)
                int32_t t2 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
                for (int wu = 0; wu < WV; ++wu) {
                    uint64_t bu = hv[wu];
                    while (bu) {
                        const int u = wu * 64 + __builtin_ctzll(bu);
                        bu &= bu - 1;
                        uint64_t hu[WV];
#pragma unroll
                        for (int w = 0; w < WV; ++w) hu[w] = R[w] & ~rows[u][w];
                        int cc = -1;  // u lies in both hv and hu
#pragma unroll
                        for (int w = 0; w < WV; ++w) cc += popc64(hv[w] & hu[w]);
                        t2 += cc;
                        if (u > v) {
                            a1 += cc;
                            a2 += cc * cc;
                            a3 += M.md[u] - 1;
                            if (cc >= 2) {
                                uint64_t X[WV];
#pragma unroll
                                for (int w = 0; w < WV; ++w) X[w] = hv[w] & hu[w] & upper_mask(u, w);
#pragma unroll
                                for (int wx = 0; wx < WV; ++wx) {
                                    while (X[wx]) {
                                        const int z = wx * 64 + __builtin_ctzll(X[wx]);
                                        X[wx] &= X[wx] - 1;
                                        int kk = 0;
#pragma unroll
                                        for (int w = 0; w < WV; ++w)
                                            if (w >= wx) kk += popc64(X[w] & ~rows[z][w]);
                                        S += 12 * kk;
                                    }
                                }
                            }
                        }
                    }
                }
                // per missing pair: 12 (cc - (m_u-1)(m_v-1)) - 4 (r-3) cc - 6 cc (cc-1)
                S += (int64_t)(18 - 4 * (r - 3)) * a1 - 6 * (int64_t)a2 - 12 * (mv - 1) * (int64_t)a3 +
                     6 * (int64_t)t2 * (mv - 2);
                // 2-paths a-v-b (a < b): 4 C4 = sum (codeg(a,b) - 1); with
                // ha = R & ~row(a), |ha & ~row(b)| = codeg(a,b) + 2 [a-b missing]
                int32_t wsum = 0;
#pragma unroll
                for (int wa = 0; wa < WV; ++wa) {
                    uint64_t ba = hv[wa];
                    while (ba) {
                        const int a0 = wa * 64 + __builtin_ctzll(ba);
                        ba &= ba - 1;
                        uint64_t ha[WV], rest[WV];
                        int corr = 0;
#pragma unroll
                        for (int w = 0; w < WV; ++w) {
                            ha[w] = R[w] & ~rows[a0][w];
                            rest[w] = hv[w] & upper_mask(a0, w);
                            corr += 2 * popc64(rest[w] & ha[w]) + popc64(rest[w]);
                        }
                        wsum -= corr;
#pragma unroll
                        for (int wb = 0; wb < WV; ++wb) {
                            if (wb < wa) continue;
                            while (rest[wb]) {
                                const int b = wb * 64 + __builtin_ctzll(rest[wb]);
                                rest[wb] &= rest[wb] - 1;
#pragma unroll
                                for (int w = 0; w < WV; ++w) wsum += popc64(ha[w] & ~rows[b][w]);
                            }
                        }
                    }
                }
                S += 3 * (int64_t)wsum;
            }
            return true;
        };

        // children of a node with l = 5 (l = 4), x in [xlo, xhi): the
        // 4-cliques (triangles) of R = P & N+(x) for each x.  A dense R is
        // counted by the wave from its missing pairs; otherwise its children
        // (x, y) join a queue in LDS and every 64 queued children are counted
        // one per lane.
        auto children_by_lanes = [&](auto wv, const auto& P, auto rows, const int16_t* col, int cn, int l, int xlo,
                                     int xhi) {
            constexpr int WV = decltype(wv)::value;
            uint64_t lsum = 0, lops = 0, usum = 0;
            int64_t S = 0;
            const int lc = l - 2;
            int qn = 0;
            // Count the queued children [base, base + cnt), cnt <= 64, one per lane.
            auto run_queue = [&](const int32_t* q, int base, int cnt) {
                if (lane < cnt) {
                    const int e = q[base + lane];
                    const int x = (e >> 8) & 0xFF, y = e & 0xFF;
                    uint64_t Q[WV];
#pragma unroll
                    for (int w = 0; w < WV; ++w) Q[w] = P[w] & rows[x][w] & rows[y][w] & upper_mask(y, w);
                    if (lc == 3) lsum += lane_triangles<WV>(rows, Q, (e >> 25) & 1, lops);
                    else lsum += lane_edges<WV>(rows, Q);
                }
            };
            // Count every queued child: a lane's work grows with |Q|, so the
            // queue is first sorted by |Q| (stable LSD passes over |Q| >> 3,
            // ballot partitions) and counted 64 at a time in that order.
            auto drain = [&]() {
                wave_sync();
                int cur = 0;
                if (qn > 64) {
                    for (int b = 19; b < 24; ++b) {
                        const int32_t* src = M.pq[cur];
                        int32_t* dst = M.pq[cur ^ 1];
                        int nz = 0;
                        for (int i0 = 0; i0 < qn; i0 += 64) {
                            const int i = i0 + lane;
                            nz += popc64(ballot(i < qn && !((src[i] >> b) & 1)));
                        }
                        int z0 = 0, o0 = nz;
                        for (int i0 = 0; i0 < qn; i0 += 64) {
                            const int i = i0 + lane;
                            const bool valid = i < qn;
                            const int e = valid ? src[i] : 0;
                            const bool one = valid && ((e >> b) & 1);
                            const uint64_t bo = ballot(one), bz = ballot(valid && !one);
                            if (valid) dst[one ? o0 + popc64(bo & lanemask_lt()) : z0 + popc64(bz & lanemask_lt())] = e;
                            z0 += popc64(bz);
                            o0 += popc64(bo);
                        }
                        wave_sync();
                        cur ^= 1;
                    }
                }
                for (int i0 = 0; i0 < qn; i0 += 64) run_queue(M.pq[cur], i0, qn - i0 < 64 ? qn - i0 : 64);
                qn = 0;
                wave_sync();
            };
            bool done = false;
            if (l == 4 && xlo == 0 && xhi >= cn) {
                const int pc = popcW(P);
                bool pd = false;
                done = pc < 4 || k4_missing(wv, P, rows, pc, true, S, usum, pd);
            }
            int xx = xlo - 1;
            while (!done) {
                int nx = -1;
#pragma unroll
                for (int w = WV - 1; w >= 0; --w) {
                    const uint64_t b = P[w] & (xx < 0 ? ~0ull : upper_mask(xx, w));
                    if (b) nx = w * 64 + __builtin_ctzll(b);
                }
                if (nx < 0 || nx >= xhi || (rule1 && col[nx] < l)) break;
                xx = nx;
                uint64_t Rx[WV];
#pragma unroll
                for (int w = 0; w < WV; ++w) Rx[w] = uni64(P[w] & rows[xx][w] & upper_mask(xx, w));
                const int rc = popcW(Rx);
                if (rc < lc + 1) continue;
                if (work) { wk_nodes += rc; wk_ops += (uint64_t)rc * WV; }
                bool rdense = false;
                if (l == 5 && k4_missing(wv, Rx, rows, rc, false, S, usum, rdense)) continue;
#pragma unroll
                for (int q = 0; q < WV; ++q) {
                    const int y = 64 * q + lane;
                    const bool act = ((Rx[q] >> lane) & 1) && !(rule1 && col[y] < l - 1);
                    const uint64_t bq = ballot(act);
                    if (act) {
                        int qy = 0;  // |Q| of the child (x, y)
#pragma unroll
                        for (int w = 0; w < WV; ++w) qy += popc64(Rx[w] & rows[y][w] & upper_mask(y, w));
                        M.pq[0][qn + popc64(bq & lanemask_lt())] = (rdense ? 1 << 25 : 0) | (qy << 16) | (xx << 8) | y;
                    }
                    qn += popc64(bq);
                }
                if (qn >= QRUN) drain();
            }
            if (qn > 0) drain();
            if (work) wk_ops += wave_sum(lops);
            const int64_t s12 = wave_sum(S);
            tacc.add((uint64_t)((int64_t)(wave_sum(lsum) + usum) + s12 / 12));
        };

        // Children of a node with l = 4 or 5 (x in [xlo, xhi)).  Classes
        // W = 2 and 3 first renumber a whole node whose candidate set fits
        // W - 1 words onto them (one narrower instance of the children and
        // leaf code per class keeps the kernel's spill space small), unless
        // the node is so small that renumbering (~6 W |P| instructions)
        // costs more than the narrower words save.
        auto count_children = [&](const uint64_t (&Pn)[W], int ln, int xlo, int xhi) {
            if constexpr (W == 2 || W == 3) {
                constexpr int WN = W - 1;
                const int p = popcW(Pn);
                if (xlo == 0 && xhi >= c && p <= 64 * WN && p >= COMPACT_MIN) {
                    uint64_t (*cr)[WN] = reinterpret_cast<uint64_t (*)[WN]>(M.crow);
                    compact_set<W, WN>(M, Pn, cr, M.ccol);
                    uint64_t Pc[WN];
                    prefix_mask<WN>(p, Pc);
                    children_by_lanes(std::integral_constant<int, WN>{}, Pc, cr, M.ccol, p, ln, 0, 64 * WN);
                    return;
                }
            }
            children_by_lanes(std::integral_constant<int, W>{}, Pn, M.rows, M.col, c, ln, xlo, xhi);
        };

        const int l0 = k - 2;
        uint64_t P0[W];
        prefix_mask<W>(c, P0);
        // A task covering the whole root may finish it in closed form; a
        // task holding only the root children with x in [x0, x1) counts
        // exactly the cliques of that part (so tasks can be listed alone).
        const bool whole = x0 == 0 && x1 >= c;
        bool active = true;
        int lq = 0;
        if (qitem >= 0) {
            // a queued node (finish() already found no closed form for it)
            lq = uniform_i32(a.squeue[qitem].l);
            if (lq == 4 || lq == 5) {
                uint64_t Pn[W];
#pragma unroll
                for (int w = 0; w < W; ++w) Pn[w] = uni64(a.squeue[qitem].P[w]);
                count_children(Pn, lq, 0, c);
                active = false;
            }
        } else if (whole) {
            u128 rootval = 0;
            active = !finish(P0, l0, rootval);
            if (!active) tacc.add(rootval);
        } else if (et && l0 >= 3) {
            // a root split over several tasks that is a clique, 2-plex or
            // 3-plex (as far as t allows): this task's part is the
            // l0-cliques whose first vertex x lies in [x0, x1), for a clique
            // sum_x C(c-1-x, l0-1), else the closed form of each later
            // neighbourhood P0 & N+(x) (a t-plex again) at l0 - 1
            int mn = 1 << 30;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int v = lane + 64 * q;
                if (v < c) {
                    int d = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) d += popc64(P0[w] & M.rows[v][w]);
                    mn = d < mn ? d : mn;
                }
            }
            const int mind = wmin_i32(mn);
            const int xe = x1 < c ? x1 : c;
            if (mind >= c - 1) {
                u128 part = 0;
                for (int x = x0; x < xe; ++x) part += binom128(c - 1 - x, l0 - 1, tacc.ovf);
                tacc.add(part);
                active = false;
            } else if (mind >= c - tpl) {
                u128 part = 0;
                bool all = true;
                for (int x = x0; x < xe && all; ++x) {
                    uint64_t Rx[W];
#pragma unroll
                    for (int w = 0; w < W; ++w) Rx[w] = uni64(P0[w] & M.rows[x][w] & upper_mask(x, w));
                    u128 v = 0;
                    all = finish(Rx, l0 - 1, v);
                    part += v;
                }
                if (all) {
                    tacc.add(part);
                    active = false;
                }
            }
        }
        if (active && qitem < 0 && (l0 == 4 || l0 == 5)) {
            count_children(P0, l0, x0, x1);
            active = false;
        }
        // hand node (Pn, ln), ln >= 4, to an idle wave through the queue
        // instead of searching it here; true when it was pushed
        // Whether waves wait for work is read from the counters (relaxed
        // loads, a round trip to L2) only every SQ_POLL_BUSY candidate nodes
        // while none wait and every SQ_POLL_HUNGRY while some do, and at
        // least every SQ_POLL_TICKS; in between the last answer stands.
        auto try_push = [&](const uint64_t (&Pn)[W], int ln) -> bool {
            if (!splitting || ln < 4) return false;
            const int pn = popcW(Pn);
            if (ln < 64 ? pn < __builtin_amdgcn_readlane(push_pmin, ln) : binom(pn, ln) < a.split_bound) return false;
            if (a.split_mode != SPLIT_FORCED) {
                if (poll_in > 0 && wall_clock64() - poll_t < SQ_POLL_TICKS) {
                    --poll_in;
                    if (!hungry) return false;
                } else {
                    poll_t = wall_clock64();
                    int hg = 0;
                    if (lane == 0) {
                        unsigned long long* sq = a.sq;
                        const unsigned long long r = sq_peek(&sq[SQ_RESERVE]), h = sq_peek(&sq[SQ_HEAD]);
                        hg = sq_peek(&sq[SQ_IDLE]) > r - h;
                    }
                    hungry = uniform_i32(__shfl(hg, 0, 64)) != 0;
                    poll_in = hungry ? SQ_POLL_HUNGRY : SQ_POLL_BUSY;
                    if (!hungry) return false;
                }
            }
            int ok = 0;
            if (lane == 0) {
                unsigned long long* sq = a.sq;
                const unsigned long long r = sq_peek(&sq[SQ_RESERVE]);
                if (r + SQ_SLACK < (unsigned long long)SQ_CAP) {
                    const unsigned long long si = sq_add(&sq[SQ_RESERVE], 1);
                    SplitItem& I = a.squeue[si];
                    I.it = (int64_t)it;
#pragma unroll
                    for (int w = 0; w < MAX_W; ++w) I.P[w] = w < W ? Pn[w] : 0;
                    I.l = ln;
                    __hip_atomic_store(&I.ready, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    sq_add(&sq[SQ_PUSHED], 1);
                    ok = 1;
                }
            }
            return uniform_i32(__shfl(ok, 0, 64)) != 0;
        };
        // depth-first search: the node being branched on lives in registers
        // (P, R, x, l); its ancestors are frames
        int sp = 0;
        uint64_t P[W], R[W];
        int x = x0 - 1, l = qitem >= 0 ? lq : l0;
#pragma unroll
        for (int w = 0; w < W; ++w) { P[w] = qitem >= 0 ? uni64(a.squeue[qitem].P[w]) : P0[w]; R[w] = 0; }
        while (active) {
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
                for (int w = 0; w < W; ++w) R[w] = uni64(P[w] & M.rows[x][w] & upper_mask(x, w));
            }
            if (y < 0) {  // node exhausted: resume the parent
                if (sp == 0) break;
                --sp;
                Frame<W>& F = FR(sp);
#pragma unroll
                for (int w = 0; w < W; ++w) { P[w] = uni64(F.P[w]); R[w] = uni64(F.R[w]); }
                x = uniform_i32(F.x);
                l = uniform_i32(F.l);
                continue;
            }
            uint64_t Pc[W];
#pragma unroll
            for (int w = 0; w < W; ++w) Pc[w] = uni64(R[w] & M.rows[y][w] & upper_mask(y, w));
            const int lc = l - 2;
            if (work) wk_ops += W;
            if (popcW(Pc) < lc) continue;
            if (rule2 && lc >= 3) {
                if (work) wk_ops += W;
                int dc = 0;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    if (q >= ncq) break;
                    bool hit = false;
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const int a0 = cs0[q] > 64 * w ? cs0[q] : 64 * w;
                        const int a1 = cs1[q] < 64 * w + 64 ? cs1[q] : 64 * w + 64;
                        if (a1 > a0) {
                            const int len = a1 - a0;
                            const uint64_t mk = (len == 64 ? ~0ull : ((1ull << len) - 1)) << (a0 - 64 * w);
                            hit |= (Pc[w] & mk) != 0;
                        }
                    }
                    dc += popc64(ballot(hit));
                }
                if (dc < lc) continue;
            }
            u128 v = 0;
            if (finish(Pc, lc, v)) { tacc.add(v); continue; }
            if (try_push(Pc, lc)) continue;
            if (lc == 4 || lc == 5) { count_children(Pc, lc, 0, c); continue; }
            if (sp >= LDS_FRAMES + (gfr ? GLOBAL_FRAMES : 0)) {
                if (lane == 0) atomicOr(a.err, ERR_DEPTH);
                continue;
            }
            if (lane == 0 || sp >= LDS_FRAMES) {
                Frame<W>& F = FR(sp);
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
    task_done:
        // a batch flags an overflow on its own graph only (top bit of the
        // graph's high word), so co-scheduled graphs keep their results
        if (tacc.ovf && lane == 0) {
            if (a.graph_total) atomicOr(&a.graph_total[2 * gi + 1], 1ull << 63);
            else atomicOr(a.err, ERR_OVERFLOW);
        }
        if (a.per_task && lane == 0) a.per_task[it] = tacc.lo();  // (no splitting with per-task counts)
        if (a.graph_total) {
            if (lane == 0 && tacc.lo()) {
                const unsigned long long old = atomicAdd(&a.graph_total[2 * gi], (unsigned long long)tacc.lo());
                if (old + tacc.lo() < old) atomicAdd(&a.graph_total[2 * gi + 1], 1ull);
            }
            if (lane == 0 && tacc.hi()) atomicAdd(&a.graph_total[2 * gi + 1], (unsigned long long)tacc.hi());
        } else {
            acc.add(tacc.v);
        }
        wave_sync();
    }
    if (work && lane == 0) {
        atomicAdd(&a.work[0], (unsigned long long)wk_tasks);
        atomicAdd(&a.work[1], (unsigned long long)wk_nodes);
        atomicAdd(&a.work[2], (unsigned long long)wk_ops);
        if (a.wave_time) {
            const unsigned long long t1 = wall_clock64();
            atomicAdd(&a.wave_time[0], t1);
            atomicMax(&a.wave_time[1], t1);
            atomicAdd(&a.wave_time[2], 1ull);
            atomicMax(&a.wave_time[3], ~(unsigned long long)t_wave0);  // earliest start, complemented
        }
    }
    if (acc.ovf && lane == 0) atomicOr(a.err, ERR_OVERFLOW);
    if (lane == 0 && acc.v) {
        const unsigned long long old = atomicAdd(&a.total[0], (unsigned long long)acc.lo());
        const unsigned long long carry = (old + acc.lo() < old) ? 1ull : 0ull;
        if (acc.hi() + carry) atomicAdd(&a.total[1], (unsigned long long)(acc.hi() + carry));
    }
}

// the split queue's counters and ready flags zeroed before a launch (a kernel,
// so that captured launch sequences hold no memset node)
__global__ void k_sq_reset(unsigned long long* sq, SplitItem* items, int64_t cap) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < SQ_WORDS) sq[i] = 0;
        items[i].ready = 0;
    }
}

hipError_t launch_sq_reset(unsigned long long* sq, SplitItem* items, hipStream_t s) {
    hipLaunchKernelGGL(k_sq_reset, dim3(64), dim3(256), 0, s, sq, items, (int64_t)SQ_CAP);
    return hipGetLastError();
}

// ---------------------------------------------------------------- EBBkC-T
// Algorithm EBBkC-T: the truss-based order pi_tau at every level.  A node is
// (P, r): vertices P of the seed's g_i and the edges among them ranked after
// r in pi_tau (r = rank of the edge added last; every edge of g_i is ranked
// after its seed, so the root is (V(g_i), -1)).  The children are the node's
// edges f = (x, y), each with the vertices of P joined to both x and y by
// edges ranked after f (Eq. edge-oriented-branching under pi_tau restricted
// to the node).  Size pruning and the clique / 2-plex terminations apply;
// the colour rules do not (the order is not colour-based).  A task keeps the
// ranks of g_i's edges in a c x c matrix in its wave's slab of device memory;
// lane j writes and reads only columns j mod 64, so no lane reads another's
// stores.  Root tasks [x0, x1) take the root edges (x, y), x < y, x in range.

template <int W>
struct TFrame {
    uint64_t P[W];
    uint64_t Y[W];  // y still to visit with the current x
    int32_t r, l, x, pad;
};

template <int W>
struct TMem {
    uint64_t rows[64 * W][W];
    TFrame<W> fr[TRUSS_FRAMES];
};

template <int W>
__global__ __launch_bounds__(256, 2) void k_search_truss(TrussArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TMem<W>& M = reinterpret_cast<TMem<W>*>(smem_raw)[threadIdx.x / 64];
    constexpr int C = 64 * W;
    int32_t* rho = a.rho + ((int64_t)blockIdx.x * 4 + threadIdx.x / 64) * (int64_t)C * C;
    const int lane = lane_id();
    const bool et = a.opts & OPT_ET, work = a.opts & OPT_WORK;
    const bool t2 = et && a.tplex != 1;
    Acc acc{0, false};
    uint64_t wk_tasks = 0, wk_nodes = 0, wk_ops = 0;

    for (;;) {
        unsigned long long it = 0;
        if (lane == 0) it = atomicAdd(a.next, 1ull);
        it = uni64(__shfl(it, 0, 64));
        if ((int64_t)it >= a.ntasks) break;
        const int64_t task = a.tasks[it];
        const int64_t slot = task_slot(task);
        const ArenaView& A = a.A;
        const int c = uniform_i32(A.seed_c[slot]);
        const int l0 = a.k - 2;
        // root ranges cover the first clique vertices 0..c-l0; here x is the
        // lower end of a clique's first edge in pi_tau, which may lie past
        // them, so the last range runs to c
        const int x0 = task_x0(task), x1 = task_x1(task) >= c - l0 + 1 ? c : task_x1(task);
        const int64_t ro = A.row_off[slot], vo = A.vtx_off[slot];
        Acc tacc{0, false};
        wk_tasks += work;
        for (int i = lane; i < c * W; i += 64) (&M.rows[0][0])[i] = A.rows[ro + i];
        wave_sync();
        // ranks of g_i's edges (entries of non-adjacent pairs are never read)
        for (int i = 0; i < c; ++i) {
            const int32_t gu = A.gid[vo + i];
            const int b = a.rp[gu], e = a.rp[gu + 1];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int j = lane + 64 * q;
                if (j < c && ((M.rows[i][q] >> lane) & 1)) {
                    const int p = lower_bound_i32(a.ci, b, e, A.gid[vo + j]);
                    rho[i * C + j] = a.erank[p];
                }
            }
        }
        if (work) wk_ops += (uint64_t)c * W;

        // nodes that need no branching: counts them (true) or returns false
        auto eval = [&](const uint64_t (&P)[W], int r, int l, u128& val) -> bool {
            const int pc = popcW(P);
            val = 0;
            if (work) wk_nodes += 1;
            if (pc < l) return true;
            if (l == 1) { val = (uint64_t)pc; return true; }
            int mn = 1 << 30, nf = 0;
            uint32_t dsum = 0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int w = lane + 64 * q;
                if ((P[q] >> lane) & 1) {
                    int d = 0;
#pragma unroll
                    for (int ww = 0; ww < W; ++ww) {
                        uint64_t bits = P[ww] & M.rows[w][ww];
                        while (bits) {
                            const int u = 64 * ww + __builtin_ctzll(bits);
                            bits &= bits - 1;
                            d += rho[u * C + w] > r;
                        }
                    }
                    mn = d < mn ? d : mn;
                    nf += d == pc - 1;
                    dsum += d;
                }
            }
            if (work) wk_ops += (uint64_t)pc * W;
            const uint64_t twoE = wsum_u32(dsum);
            if (l == 2) { val = twoE / 2; return true; }
            if (et) {
                const int mind = wmin_i32(mn);
                if (mind >= pc - 1) { val = binom128(pc, l, tacc.ovf); return true; }
                if (t2 && mind >= pc - 2) {
                    const int nfull = (int)wsum_u32((uint32_t)nf);
                    val = twoplex_count(nfull, (pc - nfull) / 2, l, tacc.ovf);
                    return true;
                }
            }
            return false;
        };
        auto write_frame = [&](int d, const uint64_t (&P)[W], int r, int l) {
            TFrame<W>& F = M.fr[d];
#pragma unroll
            for (int w = 0; w < W; ++w) { F.P[w] = P[w]; F.Y[w] = 0; }
            F.r = r;
            F.l = l;
            F.x = -1;
            wave_sync();
        };

        uint64_t P0[W];
        prefix_mask(c, P0);
        bool done = false;
        if (x0 == 0 && x1 == c) {
            u128 v = 0;
            if (eval(P0, -1, l0, v)) { tacc.add(v); done = true; }
        }
        int sp = 0;
        if (!done) write_frame(0, P0, -1, l0);
        while (!done && sp >= 0) {
            TFrame<W>& F = M.fr[sp];
            uint64_t P[W], Y[W];
#pragma unroll
            for (int w = 0; w < W; ++w) { P[w] = uni64(F.P[w]); Y[w] = uni64(F.Y[w]); }
            const int r = uniform_i32(F.r), l = uniform_i32(F.l);
            int x = uniform_i32(F.x);
            int y = -1;
#pragma unroll
            for (int w = W - 1; w >= 0; --w)
                if (Y[w]) y = 64 * w + __builtin_ctzll(Y[w]);
            if (y < 0) {  // next x of the node, and its children's y
                int nx = -1;
#pragma unroll
                for (int w = W - 1; w >= 0; --w) {
                    const uint64_t b = P[w] & upper_mask(x, w);
                    if (b) nx = 64 * w + __builtin_ctzll(b);
                }
                if (nx < 0 || (sp == 0 && (nx < x0 || nx >= x1))) {
                    if (sp == 0 && nx >= 0 && nx < x0) {  // the root starts at x0
                        F.x = x0 - 1;
                        wave_sync();
                        continue;
                    }
                    --sp;
                    continue;
                }
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const int j = lane + 64 * q;
                    bool ok = ((P[q] & M.rows[nx][q] & upper_mask(nx, q)) >> lane) & 1;
                    if (ok) ok = rho[nx * C + j] > r;
                    F.Y[q] = uni64(ballot(ok));
                }
                F.x = nx;
                wave_sync();
                if (work) wk_ops += W;
                continue;
            }
            if (lane == 0) F.Y[y >> 6] = Y[y >> 6] & (Y[y >> 6] - 1);
            wave_sync();
            // child of edge (x, y): P joined to x and y by edges ranked after it
            int rv = 0;
            if (lane == (y & 63)) rv = rho[x * C + y];
            const int rf = __shfl(rv, y & 63, 64);
            uint64_t Pc[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const int j = lane + 64 * q;
                bool in = ((P[q] & M.rows[x][q] & M.rows[y][q]) >> lane) & 1;
                if (in) in = rho[x * C + j] > rf && rho[y * C + j] > rf;
                Pc[q] = uni64(ballot(in));
            }
            if (work) wk_ops += W;
            const int lc = l - 2;
            u128 v = 0;
            if (eval(Pc, rf, lc, v)) { tacc.add(v); continue; }
            if (sp + 1 >= TRUSS_FRAMES) {
                if (lane == 0) atomicOr(a.err, ERR_DEPTH);
                break;
            }
            ++sp;
            write_frame(sp, Pc, rf, lc);
        }
        if (tacc.ovf && lane == 0) atomicOr(a.err, ERR_OVERFLOW);
        if (a.per_task && lane == 0) a.per_task[it] = tacc.lo();
        acc.add(tacc.v);
        wave_sync();
    }
    if (work && lane == 0) {
        atomicAdd(&a.work[0], (unsigned long long)wk_tasks);
        atomicAdd(&a.work[1], (unsigned long long)wk_nodes);
        atomicAdd(&a.work[2], (unsigned long long)wk_ops);
    }
    if (acc.ovf && lane == 0) atomicOr(a.err, ERR_OVERFLOW);
    if (lane == 0 && acc.v) {
        const unsigned long long old = atomicAdd(&a.total[0], (unsigned long long)acc.lo());
        const unsigned long long carry = (old + acc.lo() < old) ? 1ull : 0ull;
        if (acc.hi() + carry) atomicAdd(&a.total[1], (unsigned long long)(acc.hi() + carry));
    }
}

namespace {

template <int W, bool BUILD>
int64_t grid_blocks(int64_t ntasks, int cus, int blocks_per_cu) {
    auto kern = k_search<W, BUILD>;
    const size_t smem = 4 * sizeof(SearchMem<W>);
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess)
        return -1;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, smem) != hipSuccess) return -1;
    if (occ < 1) occ = 1;
    if (blocks_per_cu > 0 && blocks_per_cu < occ) occ = blocks_per_cu;
    // blocks_per_cu = -2: one persistent workgroup per CU fewer than fit, so a
    // launch on another stream always finds room
    if (blocks_per_cu <= -2) occ = occ > 1 ? occ - 1 : 1;
    const int64_t need = (ntasks + 3) / 4;
    // blocks_per_cu = -1: one workgroup per four tasks, not persistent, so that
    // launches on other streams get compute units as workgroups retire
    int64_t grid = blocks_per_cu == -1 ? need : (int64_t)occ * cus;
    if (grid > need) grid = need;
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    if (grid < 1) grid = 1;
    return grid;
}

template <int W, bool BUILD>
hipError_t launch_w(const SearchArgs& a, int cus, int bpc, hipStream_t s) {
    const int64_t grid = grid_blocks<W, BUILD>(a.ntasks, cus, bpc);
    if (grid < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_search<W, BUILD>), dim3((unsigned)grid), dim3(256), 4 * sizeof(SearchMem<W>), s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_search(int W, bool build, const SearchArgs& a, int cus, int bpc, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    if (build && !a.bviews) return hipErrorInvalidValue;
    switch (W * 2 + (build ? 1 : 0)) {
        case 2: return launch_w<1, false>(a, cus, bpc, s);
        case 3: return launch_w<1, true>(a, cus, bpc, s);
        case 4: return launch_w<2, false>(a, cus, bpc, s);
        case 5: return launch_w<2, true>(a, cus, bpc, s);
        case 6: return launch_w<3, false>(a, cus, bpc, s);
        case 7: return launch_w<3, true>(a, cus, bpc, s);
        case 8: return launch_w<4, false>(a, cus, bpc, s);
        case 9: return launch_w<4, true>(a, cus, bpc, s);
    }
    return hipErrorInvalidValue;
}

int64_t search_grid_waves(int W, bool build, int64_t ntasks, int cus, int bpc) {
    int64_t b = -1;
    switch (W * 2 + (build ? 1 : 0)) {
        case 2: b = grid_blocks<1, false>(ntasks, cus, bpc); break;
        case 3: b = grid_blocks<1, true>(ntasks, cus, bpc); break;
        case 4: b = grid_blocks<2, false>(ntasks, cus, bpc); break;
        case 5: b = grid_blocks<2, true>(ntasks, cus, bpc); break;
        case 6: b = grid_blocks<3, false>(ntasks, cus, bpc); break;
        case 7: b = grid_blocks<3, true>(ntasks, cus, bpc); break;
        case 8: b = grid_blocks<4, false>(ntasks, cus, bpc); break;
        case 9: b = grid_blocks<4, true>(ntasks, cus, bpc); break;
    }
    return b < 0 ? -1 : 4 * b;
}

size_t search_frame_bytes(int W) {
    switch (W) {
        case 1: return sizeof(Frame<1>);
        case 2: return sizeof(Frame<2>);
        case 3: return sizeof(Frame<3>);
        case 4: return sizeof(Frame<4>);
    }
    return 0;
}

namespace {
template <int W>
hipError_t launch_truss_w(const TrussArgs& a, int cus, hipStream_t s) {
    auto kern = k_search_truss<W>;
    const size_t smem = 4 * sizeof(TMem<W>);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    int64_t grid = (int64_t)cus * TRUSS_BLOCKS_PER_CU, need = (a.ntasks + 3) / 4;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), smem, s, a);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_search_truss(int W, const TrussArgs& a, int cus, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    switch (W) {
        case 1: return launch_truss_w<1>(a, cus, s);
        case 2: return launch_truss_w<2>(a, cus, s);
        case 3: return launch_truss_w<3>(a, cus, s);
        case 4: return launch_truss_w<4>(a, cus, s);
    }
    return hipErrorInvalidValue;
}

size_t truss_slab_bytes(int cus) {
    return (size_t)cus * TRUSS_BLOCKS_PER_CU * 4 * (size_t)(64 * MAX_W) * (64 * MAX_W) * sizeof(int32_t);
}

float k4_weight_of(int32_t dense_k4) { return dense_k4 < 0 ? 0.f : (dense_k4 == 0 ? 1.f : 0.01f * (float)dense_k4); }

hipError_t launch_binom_init(hipStream_t s) {
    hipLaunchKernelGGL(k_binom_init, dim3((BIN_N + 255) / 256), dim3(256), 0, s);
    hipLaunchKernelGGL(k_binom128_init, dim3(1), dim3(64), 0, s);
    return hipGetLastError();
}

}  // namespace ebb
