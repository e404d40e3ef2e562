"""Batched form: one fused launch per width class over the tasks of many graphs; per-graph counts
must equal the single-graph counts and the oracle, eagerly and on HIP-graph replays."""
import numpy as np
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


def mixed_graphs(count=48, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(20, 400))
        p = float(rng.uniform(0.02, 0.3))
        clique = int(rng.integers(8, 30)) if i % 4 == 0 else 0
        g = graphgen.er_planted(n, p, 1 if clique else 0, max(clique, 2), max(clique, 2), seed=1000 + i)
        k = int(rng.integers(1, 11))
        out.append((g, k))
    out.append((graphgen.cocktail_party(9), 5))
    out.append((graphgen.complete(30), 12))
    out.append((graphgen.empty(10), 3))
    out.append((configs.er_small(), 40))  # k far above tau + 2
    return out


def test_batch_matches_single_and_oracle(ebb):
    gs = mixed_graphs()
    Gs = [ebb.Graph.from_csr(g) for g, _ in gs]
    ks = [k for _, k in gs]
    want = [oracle.count(g, k) for g, k in gs]
    single = [G.count(k) for G, k in zip(Gs, ks)]
    assert single == want
    B = ebb.Batch(Gs, ks)
    assert B.run(use_graph=False) == want
    # graph replays, with eager work between them, each checked
    for rep in range(3):
        assert B.run(use_graph=True) == want, rep
        assert Gs[0].count(3) == oracle.count(gs[0][0], 3)
    B.close()
    for G in Gs:
        G.close()


def test_batch_with_split_heavy_roots_and_tuning(ebb):
    gs = [(graphgen.er_planted(300, 0.05, 1, 40, 40, seed=s), k) for s, k in zip(range(6), (6, 7, 8, 9, 10, 6))]
    Gs = [ebb.Graph.from_csr(g) for g, _ in gs]
    ks = [k for _, k in gs]
    want = [oracle.count(g, k) for g, k in gs]
    o = ebb.ebbkc_default_options()
    o.split_threshold = 500
    B = ebb.Batch(Gs, ks, options=o)
    assert B.run(use_graph=True) == want
    split, bpc, node_split = B.tune()
    assert node_split in (-1, 1 << 16, 0, 1 << 24)
    assert B.run(use_graph=True) == want
    assert B.run(use_graph=False) == want
    B.close()
    for G in Gs:
        G.close()


@pytest.mark.parametrize("ordering", [0, 1, 2])
def test_batch_tasks_that_build_their_own_subbranch(ebb, ordering):
    # batch_build = BUILD: no arena; every task builds its g_i in LDS from the graph's arrays
    # (the form for batches whose arenas would not fit device memory).  Same counts as the oracle
    # and as the arena form, eagerly and on HIP-graph replays (one task per seed when tasks build;
    # heavy roots split into ranges in the arena form).
    gs = mixed_graphs(count=40, seed=11)
    gs += [(graphgen.er_planted(300, 0.05, 1, 40, 40, seed=s), k) for s, k in zip(range(4), (6, 8, 10, 7))]
    gs += [(graphgen.er_planted(180, 0.55, 0, 2, 2, seed=21), 7), (graphgen.complete(70), 20)]
    o = ebb.ebbkc_default_options()
    o.ordering = ordering
    Gs = [ebb.Graph.from_csr(g, options=o) for g, _ in gs]
    ks = [k for _, k in gs]
    want = [oracle.count(g, k) for g, k in gs]
    for mode, split in ((ebb.BATCH_BUILD, 0), (ebb.BATCH_BUILD, 300), (ebb.BATCH_ARENA, 300)):
        ob = ebb.ebbkc_default_options()
        ob.ordering = ordering
        ob.batch_build = mode
        ob.split_threshold = split
        B = ebb.Batch(Gs, ks, options=ob)
        assert B.run(use_graph=False) == want, (mode, split)
        for rep in range(3):
            assert B.run(use_graph=True) == want, (mode, split, rep)
            assert Gs[1].count(4) == oracle.count(gs[1][0], 4)
        B.close()
    for G in Gs:
        G.close()


def test_auto_mode_builds_in_lds_without_arenas_when_they_would_not_fit(ebb):
    # graphs with no arena yet: auto mode estimates the arenas' bytes; forcing BUILD and ARENA give
    # the same counts, and a graph whose sub-branch exceeds 256 vertices is refused in BUILD mode
    gs = [(graphgen.er_planted(400, 0.1, 1, 30, 30, seed=s), 6) for s in range(5)]
    Gs = [ebb.Graph.from_csr(g) for g, _ in gs]
    ks = [k for _, k in gs]
    want = [oracle.count(g, k) for g, k in gs]
    B = ebb.Batch(Gs, ks)  # auto: these arenas fit easily
    assert B.run() == want
    B.close()
    wide = ebb.Graph.from_csr(graphgen.complete(300))
    ob = ebb.ebbkc_default_options()
    ob.batch_build = ebb.BATCH_BUILD
    with pytest.raises(ebb.EbbkcError) as ei:
        ebb.Batch([wide], [5], options=ob)
    assert ei.value.status == ebb.E_WIDTH
    wide.close()
    for G in Gs:
        G.close()
