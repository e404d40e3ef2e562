"""Runtime splitting of search nodes over waves through the device queue (root sub-branches and
their subtrees are independent, Section 6.2 (7)): counts equal the oracle's (or the closed form of
complete multipartite graphs) with splitting forced at every depth (every node with l >= 4 handed
to the queue while it has room), on demand with the smallest bound, by default and off; the
counters report the nodes handed over; batches split the same way."""
import itertools

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


def elementary(parts, k):
    # e_k of the part sizes: the k-cliques of a complete multipartite graph
    e = [1] + [0] * k
    for a in parts:
        for j in range(k, 0, -1):
            e[j] += e[j - 1] * a
    return e[k]


# (name, graph, k values, part sizes of a complete multipartite graph, whether searches there branch
# on nodes with l >= 4 that no closed form ends, so that forced splitting must hand some over)
CASES = [
    ("er200", lambda: graphgen.er(200, 0.5, seed=4), range(6, 12), None, True),
    ("rmat12", lambda: configs.rmat_scale(12), range(7, 12), None, True),
    ("multipartite", lambda: graphgen.complete_multipartite([3] * 16), range(6, 11), [3] * 16, True),
    ("planted", lambda: graphgen.er_planted(400, 0.08, 3, 24, 30, seed=8), range(6, 11), None, False),
]


@pytest.mark.parametrize("name,make,ks,parts,branches", CASES, ids=[c[0] for c in CASES])
def test_counts_with_node_splitting(ebb, name, make, ks, parts, branches):
    g = make()
    want = {k: (elementary(parts, k) if parts else oracle.count(g, k)) for k in ks}
    for mode in (1, 2, 0, -1):
        o = ebb.ebbkc_default_options()
        o.node_split = mode
        o.count_work = 1
        G = ebb.Graph.from_csr(g, options=o)
        pushed = 0
        for k in ks:
            print(f"case split {name} mode={mode} k={k}", flush=True)
            assert G.count(k) == want[k], (mode, k)
            pushed += G.last_work()[3]
        if mode == 1 and branches:
            assert pushed > 0  # forced: nodes went through the queue
        if mode == -1:
            assert pushed == 0
        G.close()


def test_batch_with_forced_splitting(ebb):
    gs = [(graphgen.er(200, 0.5, seed=4), 9), (configs.rmat_scale(12), 9), (graphgen.er_planted(400, 0.08, 3, 24, 30, seed=8), 8),
          (graphgen.complete_multipartite([3] * 16), 8)]
    want = [oracle.count(g, k) if i < 3 else elementary([3] * 16, k) for i, (g, k) in enumerate(gs)]
    Gs = [ebb.Graph.from_csr(g) for g, _ in gs]
    for mode, build in itertools.product((1, 0), (ebb.BATCH_ARENA, ebb.BATCH_BUILD)):
        o = ebb.ebbkc_default_options()
        o.node_split = mode
        o.batch_build = build
        B = ebb.Batch(Gs, [k for _, k in gs], options=o)
        assert B.run(use_graph=False) == want, (mode, build)
        for rep in range(2):
            assert B.run(use_graph=True) == want, (mode, build, rep)
        B.close()
    for G in Gs:
        G.close()
