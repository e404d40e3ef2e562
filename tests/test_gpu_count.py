"""Parity of the HIP path (through the C-ABI) with the CPU oracle: counts bit-exact.

Small and medium graphs are compared element by element (per-edge supports, truss levels, ranks,
sub-branch sizes) and count by count; the headline R-MAT graph is compared against stored oracle
values (tests/golden/, written by tests/golden/make_golden.py from the oracle alone) and on sampled
seeds whose per-seed counts the oracle computes one by one.
"""
import json
import math
import os

import numpy as np
import pytest

import graphgen
import oracle
from graphgen import configs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ebb():
    import torch
    import paper_2311_13798_amd as m
    torch.cuda.set_device(0)
    m.load_library()
    return m


def opts(ebb, **kw):
    o = ebb.ebbkc_default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def small_graphs():
    fx = json.load(open(os.path.join(GOLDEN, "appendix_b.json")))
    out = [
        ("appendix_b", graphgen.from_edges(4, fx["edges"])),
        ("er_small", configs.er_small()),
        ("rmat10", graphgen.rmat(10, 16, seed=3)),
        ("rmat12", graphgen.rmat(12, 16, seed=1)),
        ("cl_20k", configs.cl_planted(20000, nplant=6)),
        ("er_planted", graphgen.er_planted(500, 0.08, 2, 20, 40, 5)),
        ("K9", graphgen.complete(9)),
        ("K_8_8", graphgen.complete_multipartite([8, 8])),
        ("cocktail12", graphgen.cocktail_party(12)),
        ("single_edge", graphgen.from_edges(5, [[1, 3]])),
        ("empty", graphgen.empty(7)),
    ]
    return out


@pytest.mark.parametrize("name,g", small_graphs(), ids=lambda x: x if isinstance(x, str) else "")
def test_prepare_arrays_match_oracle(ebb, name, g):
    print(f"case prepare {name} n={g.n} m={g.m}", flush=True)
    G = ebb.Graph.from_csr(g)
    tr = oracle.truss_levelsync(g)
    assert G.info.m == g.m
    assert G.info.tau == tr["tau"]
    assert G.info.rounds == tr["rounds"]
    if g.m:
        assert (G.export(ebb.ARR_SUPPORT) == oracle.edge_support(g)).all()
        assert (G.export(ebb.ARR_LEVEL) == tr["level"]).all()
        assert (G.export(ebb.ARR_RANK) == tr["rank"]).all()
        assert (G.export(ebb.ARR_SUBSIZE) == oracle.seed_sizes(g, tr["rank"])).all()
    G.close()


@pytest.mark.parametrize("name,g", small_graphs(), ids=lambda x: x if isinstance(x, str) else "")
def test_counts_match_oracle(ebb, name, g):
    G = ebb.Graph.from_csr(g)
    kmax = min(G.info.tau + 4, 14)
    for k in range(1, kmax + 1):
        print(f"case count {name} k={k}", flush=True)
        assert G.count(k) == oracle.count(g, k), (name, k)
    G.close()


def test_counts_random_graphs(ebb):
    rng = np.random.default_rng(2024)
    for trial in range(150):
        n = int(rng.integers(2, 60))
        p = float(rng.uniform(0.05, 0.95))
        g = graphgen.er(n, p, seed=7000 + trial)
        G = ebb.Graph.from_csr(g)
        for k in range(3, min(n, 12) + 1):
            want = oracle.count(g, k, threads=1)
            got = G.count(k)
            assert got == want, (trial, n, p, k, got, want)
        G.close()


def test_host_input_path(ebb):
    g = graphgen.rmat(9, 8, seed=11)
    G = ebb.Graph.from_csr(g, device=False)
    for k in (3, 4, 5):
        assert G.count(k) == oracle.count(g, k)
    G.close()


@pytest.mark.parametrize("toggle", [dict(early_termination=0), dict(t_plex=1), dict(rule1=0), dict(rule2=0),
                                    dict(rule1=0, rule2=0, early_termination=0), dict(blocks_per_cu=1)])
def test_switches_do_not_change_counts(ebb, toggle):
    for g in [graphgen.er_planted(300, 0.1, 3, 15, 30, 9), graphgen.cocktail_party(10), configs.er_small(),
              graphgen.rmat(11, 16, seed=2)]:
        G = ebb.Graph.from_csr(g, options=opts(ebb, **toggle))
        for k in range(3, 10):
            assert G.count(k) == oracle.count(g, k), (toggle, g.name, k)
        G.close()


@pytest.mark.parametrize("p", [3, 8, 20, 31, 32, 33, 60])
def test_two_plex_closed_form(ebb, p):
    g = graphgen.cocktail_party(p)
    G = ebb.Graph.from_csr(g)
    for k in range(1, min(p, 14) + 2):
        assert G.count(k) == math.comb(p, k) * 2 ** k, (p, k)
    G.close()


@pytest.mark.parametrize("size", [30, 63, 64, 65, 66, 127, 128, 130, 191, 192, 194, 240])
def test_width_classes_on_planted_cliques(ebb, size):
    # one planted clique on a sparse background: sub-branches near every bitmap width boundary
    g = graphgen.er_planted(max(400, 2 * size), 0.01, 1, size, size, seed=size)
    G = ebb.Graph.from_csr(g)
    for k in (3, 4, 5, 8, size - 1, size, size + 1):
        if k < 3:
            continue
        want = oracle.count(g, k)
        assert G.count(k) == want, (size, k)
    G.close()


def test_k_edge_cases(ebb):
    g = configs.er_small()
    G = ebb.Graph.from_csr(g)
    assert G.count(1) == g.n
    assert G.count(2) == g.m
    assert G.count(G.info.tau + 3) == 0
    with pytest.raises(ebb.EbbkcError) as ei:
        G.count(0)
    assert ei.value.status == ebb.E_K_RANGE
    G.close()
    E = ebb.Graph.from_csr(graphgen.empty(5))
    assert E.count(3) == 0 and E.count(1) == 5 and E.count(2) == 0
    E.close()


def test_bad_csr_is_rejected(ebb):
    g = graphgen.er(30, 0.3, seed=1)
    h = graphgen.Graph(g.n, g.row_ptr.copy(), g.col_idx.copy())
    h.col_idx[h.row_ptr[5]] = 5  # self-loop
    with pytest.raises(ebb.EbbkcError) as ei:
        ebb.Graph.from_csr(h)
    assert ei.value.status == ebb.E_BAD_CSR
    h = graphgen.Graph(g.n, g.row_ptr.copy(), g.col_idx.copy())
    r = h.row_ptr[3]
    h.col_idx[r], h.col_idx[r + 1] = h.col_idx[r + 1], h.col_idx[r]
    with pytest.raises(ebb.EbbkcError):
        ebb.Graph.from_csr(h)
    h = graphgen.Graph(g.n, g.row_ptr.copy(), g.col_idx.copy())
    h.row_ptr[4] = h.row_ptr[5] + 1  # non-monotone offsets
    with pytest.raises(ebb.EbbkcError):
        ebb.Graph.from_csr(h)


def test_relabelling_invariance(ebb):
    g = graphgen.rmat(12, 16, seed=9)
    h = graphgen.permute(g, seed=5)
    G, H = ebb.Graph.from_csr(g), ebb.Graph.from_csr(h)
    for k in (3, 5, 7, 9):
        assert G.count(k) == H.count(k)
    G.close()
    H.close()


def test_rank_ranges_partition_the_count(ebb):
    g = graphgen.rmat(12, 16, seed=4)
    G = ebb.Graph.from_csr(g)
    m = G.info.m
    cuts = sorted(set([0, m] + list(np.random.default_rng(1).integers(0, m, 7))))
    for k in (3, 5, 7):
        parts = sum(G.count_range(k, a, b) for a, b in zip(cuts[:-1], cuts[1:]))
        assert parts == G.count(k) == oracle.count(g, k)
    # single-seed ranges equal the oracle's per-seed counts
    tr = oracle.truss_levelsync(g)
    eids = np.argsort(tr["rank"])[-40:]
    want = oracle.seed_counts(g, tr["rank"], 5, eids)
    for e, w in zip(eids, want):
        r = int(tr["rank"][e])
        assert G.count_range(5, r, r + 1) == int(w)
    G.close()


def test_er_small_golden(ebb):
    fx = json.load(open(os.path.join(GOLDEN, "er_small.json")))
    g = configs.er_small()
    assert g.sha256() == fx["sha256"]
    G = ebb.Graph.from_csr(g)
    for k, v in fx["counts"].items():
        assert G.count(int(k)) == v
    G.close()


def elementary_symmetric(parts, k):
    e = [1] + [0] * k
    for a in parts:
        for j in range(k, 0, -1):
            e[j] += e[j - 1] * a
    return e[k]


@pytest.mark.parametrize("parts,kmax", [([4] * 12, 12), ([5, 4, 3, 6, 2, 7, 4, 5, 3, 3], 10), ([6] * 20, 8),
                                        ([4] * 45, 7), ([3] * 80, 6), ([2] * 30 + [5] * 12, 8)],
                         ids=["4x12", "mixed10", "6x20", "4x45", "3x80", "2x30_5x12"])
def test_complete_multipartite_closed_form(ebb, parts, kmax):
    # the missing pairs form disjoint cliques (triangles, diamonds and K4s among them for parts
    # of 4 and more): N_k is the k-th elementary symmetric polynomial of the part sizes
    g = graphgen.complete_multipartite(parts)
    G = ebb.Graph.from_csr(g)
    for k in range(1, kmax + 1):
        print(f"case multipartite {len(parts)} parts k={k}", flush=True)
        assert G.count(k) == elementary_symmetric(parts, k), (parts, k)
    G.close()


@pytest.mark.parametrize("n,pm,kmax", [(30, 0.05, 9), (40, 0.15, 8), (40, 0.3, 8), (70, 0.03, 8), (70, 0.1, 8),
                                      (130, 0.05, 6), (200, 0.04, 6), (250, 0.03, 5)])
def test_near_cliques_match_oracle(ebb, n, pm, kmax):
    # the complement of a sparse random graph: every candidate set is dense, so 4-cliques are
    # counted from the missing pairs; also with that evaluation switched off
    h = graphgen.er(n, pm, seed=int(1000 * pm) + n)
    edges = set(map(tuple, h.edges().tolist()))
    g = graphgen.from_edges(n, [[a, b] for a in range(n) for b in range(a + 1, n) if (a, b) not in edges])
    G = ebb.Graph.from_csr(g)
    G0 = ebb.Graph.from_csr(g, options=opts(ebb, dense_k4=-1))
    for k in range(3, kmax + 1):
        print(f"case near-clique n={n} pm={pm} k={k}", flush=True)
        want = oracle.count(g, k)
        assert G.count(k) == want, (n, pm, k)
        assert G0.count(k) == want, (n, pm, k)
    G.close()
    G0.close()
