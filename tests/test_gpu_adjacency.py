"""Sub-branch builds by pair tests against an adjacency bitmap of G (graphs up to adj_max_n vertices)
and by scanning the members' rows: both give g_i of Eq. edge-oriented-branching, so sub-branch sizes
(against the oracle's seed_sizes), per-seed counts, whole counts and batched counts with tasks that
build in LDS agree with the oracle under either path, at the bitmap's word boundaries too."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ebb():
    import torch
    import paper_2311_13798_amd as m
    torch.cuda.set_device(0)
    m.load_library()
    return m


def cases():
    return [
        ("er300_p02", graphgen.er_planted(300, 0.2, 0, 2, 2, seed=5), (3, 4, 5, 6, 7)),
        ("er1000_p01_planted", graphgen.er_planted(1000, 0.1, 1, 40, 40, seed=6), (4, 6, 9, 12)),
        ("er129_dense", graphgen.er_planted(129, 0.6, 0, 2, 2, seed=7), (5, 8, 10)),
        ("er64_words", graphgen.er_planted(64, 0.5, 0, 2, 2, seed=8), (4, 6)),
        ("complete70", graphgen.complete(70), (5, 62)),
        ("cocktail12", graphgen.cocktail_party(12), (4, 7)),
    ]


def opts(ebb, adj):
    o = ebb.ebbkc_default_options()
    o.adj_max_n = adj
    return o


@pytest.mark.parametrize("name,g,ks", cases(), ids=[c[0] for c in cases()])
def test_pair_build_and_scan_build_agree_with_the_oracle(ebb, name, g, ks):
    print(f"case {name} n={g.n}", flush=True)
    tr = oracle.truss_levelsync(g)
    want_sizes = oracle.seed_sizes(g, tr["rank"])
    want = {k: oracle.count(g, k) for k in ks}
    rng = np.random.default_rng(1)
    eids = np.sort(rng.choice(g.m, size=min(40, g.m), replace=False)).astype(np.int64)
    for adj in (0, -1, g.n, g.n - 1):  # default (bitmap), scan, bound at n (bitmap), just below n (scan)
        G = ebb.Graph.from_csr(g, options=opts(ebb, adj))
        assert (G.export(ebb.ARR_RANK) == tr["rank"]).all(), adj
        assert (G.export(ebb.ARR_SUBSIZE) == want_sizes).all(), adj
        for k in ks:
            assert G.count(k) == want[k], (adj, k)
        k = ks[len(ks) // 2]
        out = np.zeros(eids.size, np.uint64)
        ebb.ebbkc_count_seeds(G.handle, k, eids, out)
        assert (out == oracle.seed_counts(g, tr["rank"], k, eids)).all(), (adj, k)
        G.close()


def test_batches_that_build_in_lds_under_either_path(ebb):
    rng = np.random.default_rng(4)
    gs = [(graphgen.er_planted(int(rng.integers(60, 700)), float(rng.uniform(0.05, 0.3)), i % 2, 25, 25,
                               seed=70 + i), int(rng.integers(3, 11))) for i in range(24)]
    want = [oracle.count(g, k) for g, k in gs]
    for adj in (0, -1):
        Gs = [ebb.Graph.from_csr(g, options=opts(ebb, adj)) for g, _ in gs]
        ob = opts(ebb, adj)
        ob.batch_build = ebb.BATCH_BUILD
        B = ebb.Batch(Gs, [k for _, k in gs], options=ob)
        assert B.run(use_graph=False) == want, adj
        assert B.run(use_graph=True) == want, adj
        if adj == 0:  # the tuner's settings all give these counts, and so does its choice
            B.tune()
            assert B.run(use_graph=True) == want
        B.close()
        for G in Gs:
            G.close()


def test_adjacency_bound_is_validated(ebb):
    g = graphgen.complete(8)
    for bad in (-2, 32769):
        with pytest.raises(ebb.EbbkcError) as ei:
            ebb.Graph.from_csr(g, options=opts(ebb, bad))
        assert ei.value.status == ebb.E_INVALID_ARG
    G = ebb.Graph.from_csr(g, options=opts(ebb, 32768))
    assert G.count(5) == 56
    G.close()
