"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each check below is computed independently of the function it pins: brute force over subsets,
closed forms of graph families, the paper's worked examples (tests/golden/), the definition of a
k-truss by exhaustive search, and properties the paper proves (Lemma tau < delta, every k-clique
listed exactly once).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import graphgen
import oracle
from graphgen import configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def dense_adj(g):
    A = np.zeros((g.n, g.n), dtype=np.int64)
    src = np.repeat(np.arange(g.n), g.degrees())
    A[src, g.col_idx] = 1
    return A


def py_cliques(g, k):
    """All k-cliques by itertools over k-subsets (tiny graphs only)."""
    A = dense_adj(g)
    out = []
    for c in itertools.combinations(range(g.n), k):
        if all(A[a, b] for a, b in itertools.combinations(c, 2)):
            out.append(c)
    return out


def elem_sym(parts, k):
    e = [1] + [0] * k
    for a in parts:
        for j in range(k, 0, -1):
            e[j] += e[j - 1] * a
    return e[k]


# ------------------------------------------------------------------ counting

def test_vbb_matches_brute_force_on_random_tiny_graphs():
    rng = np.random.default_rng(7)
    for trial in range(2000):
        n = int(rng.integers(0, 17))
        p = float(rng.uniform(0.0, 1.0))
        g = graphgen.er(n, p, seed=1000 + trial)
        for k in range(1, n + 2):
            b = oracle.count_brute(g, k)
            assert oracle.count(g, k, threads=1) == b, (trial, n, p, k)
            if k >= 3 and trial % 4 == 0:
                assert oracle.count(g, k, threads=2, shortcut=False) == b


def test_brute_force_matches_itertools_definition():
    for trial in range(60):
        g = graphgen.er(9, 0.2 + 0.01 * trial, seed=77 + trial)
        for k in range(1, 8):
            assert oracle.count_brute(g, k) == len(py_cliques(g, k))


@pytest.mark.parametrize("n", [1, 2, 5, 13, 40, 64, 67])
def test_complete_graph_binomials(n):
    g = graphgen.complete(n)
    for k in range(1, n + 2):
        assert oracle.count(g, k) == math.comb(n, k)


def test_overflow_is_reported_not_wrapped():
    g = graphgen.complete(70)
    assert math.comb(70, 35) > 2**64 - 1
    with pytest.raises(oracle.OracleError) as ei:
        oracle.count(g, 35)
    assert ei.value.code == oracle.OVERFLOW
    with pytest.raises(oracle.OracleError):
        oracle.binom(70, 35)
    assert oracle.binom(67, 33) == math.comb(67, 33)


@pytest.mark.parametrize("parts", [[3, 3, 3], [1, 2, 3, 4, 5], [5, 1, 1, 7], [2] * 9, [10, 10]])
def test_complete_multipartite_elementary_symmetric(parts):
    g = graphgen.complete_multipartite(parts)
    for k in range(1, len(parts) + 2):
        assert oracle.count(g, k) == elem_sym(parts, k)


@pytest.mark.parametrize("p", [1, 3, 6, 11])
def test_cocktail_party(p):
    g = graphgen.cocktail_party(p)
    for k in range(1, p + 2):
        assert oracle.count(g, k) == math.comb(p, k) * 2**k


def test_disjoint_cliques():
    sizes = [3, 7, 12, 20]
    g = graphgen.disjoint_cliques(sizes)
    for k in range(1, 22):
        assert oracle.count(g, k) == sum(math.comb(s, k) for s in sizes)


def test_complete_bipartite_has_no_triangles_tau_zero():
    # Section 4.2 (discussion of tau): K_{p,p} has delta = p and tau = 0.
    p = 9
    g = graphgen.complete_multipartite([p, p])
    assert oracle.count(g, 3) == 0
    assert oracle.degeneracy(g)[1] == p
    t = oracle.truss_levelsync(g)
    assert t["tau"] == 0
    assert (oracle.edge_support(g) == 0).all()


def test_k3_equals_trace_of_cube_over_six():
    for g in [configs.er_small(), graphgen.er(300, 0.1, 3), graphgen.rmat(10, 8, seed=2)]:
        A = dense_adj(g).astype(np.float64)
        tr = int(round(np.trace(A @ A @ A)))
        assert tr % 6 == 0
        n3 = oracle.count(g, 3)
        assert n3 == tr // 6
        assert int(oracle.edge_support(g).sum()) == 3 * n3


def test_relabelling_invariance():
    g = graphgen.rmat(11, 8, seed=5)
    h = graphgen.permute(g, seed=99)
    for k in (3, 4, 5, 6):
        assert oracle.count(g, k) == oracle.count(h, k)


def test_two_plex_example_counts():
    fx = load("two_plex_example.json")
    n = fx["n"]
    non = {tuple(e) for e in fx["non_edges"]}
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if (a, b) not in non]
    g = graphgen.from_edges(n, edges)
    for k, v in fx["derived"]["N"].items():
        assert oracle.count(g, int(k)) == v
        assert oracle.count_brute(g, int(k)) == v


# ------------------------------------------------------------------ listing

def py_checksums(tuples, k):
    M = (1 << 64) - 1

    def sm(x):
        z = (x + 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    ho = hu = 0
    for i, t in enumerate(tuples):
        h = k
        for a in t:
            h = sm(h ^ int(a))
        hu = (hu + h) & M
        ho = (ho + sm(h ^ sm(i))) & M
    return ho, hu


def test_listing_is_the_sorted_set_of_cliques():
    for trial in range(40):
        g = graphgen.er(12, 0.3 + 0.015 * trial, seed=500 + trial)
        for k in range(1, 7):
            c, ho, hu, tup = oracle.list_lex(g, k, threads=2)
            ref = py_cliques(g, k)
            assert c == len(ref)
            assert [tuple(t) for t in tup.tolist()] == ref  # itertools order is lexicographic
            assert (ho, hu) == py_checksums(ref, k)


def test_listing_on_small_workload():
    g = configs.er_small()
    A = dense_adj(g)
    for k in (3, 4):
        c, ho, hu, tup = oracle.list_lex(g, k)
        assert c == oracle.count(g, k)
        if c:
            assert (np.diff(tup, axis=1) > 0).all()
            keys = [tuple(t) for t in tup.tolist()]
            assert keys == sorted(set(keys))
            for t in tup:
                assert all(A[a, b] for a, b in itertools.combinations(t, 2))
        assert (ho, hu) == py_checksums(tup.tolist(), k)
    c2, *_ = oracle.list_lex(g, 4, want_tuples=False)
    assert c2 == oracle.count(g, 4)


def test_tuple_hash_matches_definition():
    t = [3, 17, 99, 1 << 20]
    assert oracle.tuple_hash(t) == py_checksums([t], 4)[1]


# ------------------------------------------------------------------ truss ordering

def brute_trussness(g):
    """Trussness of every edge by definition: the largest t such that some edge subset H
    containing e has every edge of H in >= t-2 triangles of H (m <= 14)."""
    eu, ev = oracle.edge_list(g)
    m = len(eu)
    E = list(zip(eu.tolist(), ev.tolist()))
    idx = {e: i for i, e in enumerate(E)}
    tri = []
    for i, (a, b) in enumerate(E):
        for w in range(g.n):
            if w in (a, b):
                continue
            f, h = idx.get((min(a, w), max(a, w))), idx.get((min(b, w), max(b, w)))
            if f is not None and h is not None:
                tri.append((i, f, h))
    best = [2] * m
    for mask in range(1, 1 << m):
        sup = [0] * m
        for (i, f, h) in tri:
            if mask >> i & 1 and mask >> f & 1 and mask >> h & 1:
                sup[i] += 1
        members = [i for i in range(m) if mask >> i & 1]
        t = min(sup[i] for i in members) + 2
        for i in members:
            best[i] = max(best[i], t)
    return np.array(best)


def test_levelsync_level_is_trussness_minus_two():
    rng = np.random.default_rng(3)
    done = 0
    for trial in range(400):
        n = int(rng.integers(3, 8))
        g = graphgen.er(n, float(rng.uniform(0.3, 1.0)), seed=9000 + trial)
        if g.m == 0 or g.m > 13:
            continue
        t = oracle.truss_levelsync(g)
        assert (t["level"] == brute_trussness(g) - 2).all(), trial
        done += 1
    assert done > 100


def test_sequential_peel_running_max_is_level():
    for seed in range(30):
        g = graphgen.er(40, 0.25, seed=seed)
        order, peel = oracle.truss_sequential(g)
        run = np.maximum.accumulate(peel[order])
        lev = np.empty_like(run)
        lev[order] = run
        assert (lev == oracle.truss_levelsync(g)["level"]).all()


def test_sequential_peel_value_is_subbranch_size():
    # Eq. tau: |V(g_i)| is the common-neighbour count of e_i in the graph of
    # the edges not yet removed -- exactly what the greedy rule minimises.
    for seed in range(20):
        g = graphgen.er(60, 0.2, seed=100 + seed)
        order, peel = oracle.truss_sequential(g)
        rank = np.empty(len(order), np.int32)
        rank[order] = np.arange(len(order), dtype=np.int32)
        assert (oracle.seed_sizes(g, rank) == peel).all()


@pytest.mark.parametrize("maker", [lambda: configs.er_small(), lambda: graphgen.rmat(12, 16, seed=4),
                                   lambda: graphgen.chung_lu(20000, 2.1, 30.0, 4, 30, 60, seed=2),
                                   lambda: graphgen.er_planted(400, 0.05, 1, 25, 25, 8)])
def test_levelsync_invariants(maker):
    g = maker()
    t = oracle.truss_levelsync(g)
    m = g.m
    rank, level, rnd = t["rank"], t["level"], t["round"]
    assert sorted(rank.tolist()) == list(range(m))
    order = np.argsort(rank)
    # ranks follow (round, edge id)
    key = rnd[order].astype(np.int64) * (m + 1) + order
    assert (np.diff(key) > 0).all()
    assert (np.diff(level[order]) >= 0).all()
    c = oracle.seed_sizes(g, rank)
    assert (c <= level).all()
    assert t["tau"] == (level.max() if m else 0)
    assert c.max(initial=0) <= t["tau"]
    # Lemma (tau < delta), Section 4.2
    if m:
        assert t["tau"] < oracle.degeneracy(g)[1]
    assert int(c.sum()) == oracle.count(g, 3)


def test_appendix_b_example():
    fx = load("appendix_b.json")
    g = graphgen.from_edges(4, fx["edges"])
    d = fx["derived"]
    for k, v in d["N"].items():
        assert oracle.count(g, int(k)) == v
    assert oracle.degeneracy(g)[1] == d["delta"]
    t = oracle.truss_levelsync(g)
    assert t["tau"] == d["tau"]
    eu, ev = oracle.edge_list(g)
    eid = {(a, b): i for i, (a, b) in enumerate(zip(eu.tolist(), ev.tolist()))}
    printed = [eid[tuple(e)] for e in fx["printed_truss_order"]]
    rank = np.empty(5, np.int32)
    rank[printed] = np.arange(5)
    assert oracle.seed_sizes(g, rank)[printed].tolist() == d["subbranch_sizes_printed_order"]
    lvl_order = np.argsort(t["rank"])
    assert oracle.seed_sizes(g, t["rank"])[lvl_order].tolist() == d["subbranch_sizes_printed_order"]


# ------------------------------------------------------------------ exactly-once partition

def test_edge_branching_partition_counts_every_clique_once():
    rng = np.random.default_rng(11)
    for trial in range(30):
        g = graphgen.er(int(rng.integers(10, 40)), float(rng.uniform(0.2, 0.8)), seed=300 + trial)
        m = g.m
        rankings = [oracle.truss_levelsync(g)["rank"], rng.permutation(m).astype(np.int32)]
        order, _ = oracle.truss_sequential(g)
        r = np.empty(m, np.int32)
        r[order] = np.arange(m)
        rankings.append(r)
        for k in range(3, 8):
            want = oracle.count(g, k)
            for rank in rankings:
                assert int(oracle.seed_counts(g, rank, k).sum()) == want, (trial, k)


# ------------------------------------------------------------------ input validation

def test_validation_rejects_malformed_csr():
    g = graphgen.er(30, 0.3, seed=1)
    assert oracle.validate(g) == 0
    bad = []
    h = graphgen.Graph(g.n, g.row_ptr.copy(), g.col_idx.copy())
    r = h.row_ptr[3]
    h.col_idx[r], h.col_idx[r + 1] = h.col_idx[r + 1], h.col_idx[r]  # unsorted row
    bad.append(h)
    h = graphgen.Graph(g.n, g.row_ptr.copy(), g.col_idx.copy())
    h.col_idx[h.row_ptr[5]] = 5  # self-loop
    bad.append(h)
    h = graphgen.Graph(g.n, g.row_ptr.copy(), g.col_idx.copy())
    h.col_idx[h.row_ptr[6] + 1] = h.col_idx[h.row_ptr[6]]  # duplicate
    bad.append(h)
    # asymmetric: drop one direction of an edge
    e = g.edges()[0]
    keep = np.ones(g.nnz, bool)
    pos = g.row_ptr[e[0]] + np.searchsorted(g.col_idx[g.row_ptr[e[0]]:g.row_ptr[e[0] + 1]], e[1])
    keep[pos] = False
    rp = g.row_ptr.copy()
    rp[e[0] + 1:] -= 1
    bad.append(graphgen.Graph(g.n, rp, g.col_idx[keep]))
    for b in bad:
        assert oracle.validate(b) == oracle.BAD_CSR
