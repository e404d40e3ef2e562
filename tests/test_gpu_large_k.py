"""Counts near the maximum clique size: exact 128-bit counts (ebbkc_count128) pinned by closed forms
computed with Python integers (C(n, k) for K_n, sums over disjoint cliques, C(p, k) 2^k for cocktail
parties), the 64-bit call's overflow error past 2^64, the 128-bit call's past 2^128, and the maximum
clique size omega (ebbkc_max_clique_size) against closed forms and the oracle."""
import math

import pytest

import graphgen
import oracle
from graphgen import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ebb():
    import torch
    import paper_2311_13798_amd as m
    torch.cuda.set_device(0)
    m.load_library()
    return m


@pytest.mark.parametrize("n", [70, 100, 130, 190, 250])
def test_complete_graphs_128_bit(ebb, n):
    G = ebb.Graph.from_csr(graphgen.complete(n))
    for k in sorted({3, 5, 20, n // 3, n // 2, n - 5, n - 1, n, n + 1}):
        want = math.comb(n, k)
        print(f"case K{n} k={k}", flush=True)
        if want >= 1 << 128:
            with pytest.raises(ebb.EbbkcError) as ei:
                G.count128(k)
            assert ei.value.status == ebb.E_OVERFLOW
            continue
        assert G.count128(k) == want, (n, k)
        if want >= 1 << 64:
            with pytest.raises(ebb.EbbkcError) as ei:
                G.count(k)
            assert ei.value.status == ebb.E_OVERFLOW
        else:
            assert G.count(k) == want
    assert G.max_clique_size() == n
    G.close()


def test_disjoint_cliques_128_bit(ebb):
    sizes = [40, 70, 90, 120, 9]
    G = ebb.Graph.from_csr(graphgen.disjoint_cliques(sizes))
    for k in (3, 10, 35, 45, 60, 89, 90, 91, 120):
        assert G.count128(k) == sum(math.comb(s, k) for s in sizes), k
    assert G.max_clique_size() == 120
    G.close()


@pytest.mark.parametrize("p", [40, 70, 100])
def test_cocktail_party_128_bit(ebb, p):
    # every vertex misses exactly one other: the 2-plex closed form at every node
    G = ebb.Graph.from_csr(graphgen.cocktail_party(p))
    for k in (4, p // 2, p - 1, p):
        want = math.comb(p, k) * 2 ** k
        if want >= 1 << 128:
            continue
        assert G.count128(k) == want, (p, k)
    assert G.max_clique_size() == p
    G.close()


@pytest.mark.parametrize("name,g", [("er_small", configs.er_small()), ("rmat10", graphgen.rmat(10, 16, seed=3)),
                                    ("er_planted", graphgen.er_planted(400, 0.03, 2, 15, 22, 7)),
                                    ("single_edge", graphgen.from_edges(5, [[1, 3]])), ("empty", graphgen.empty(4))],
                         ids=lambda x: x if isinstance(x, str) else "")
def test_max_clique_size_matches_the_oracle(ebb, name, g):
    G = ebb.Graph.from_csr(g)
    omega = G.max_clique_size()
    if g.m == 0:
        assert omega == (1 if g.n else 0)
    else:
        assert oracle.count(g, omega) > 0 and oracle.count(g, omega + 1) == 0
    G.close()
