"""ebbkc_count_noalloc: the count with no allocation (a fixed per-device scratch buffer) equals
ebbkc_count on the same handle, on consecutive calls whose second input is smaller than the first
(the buffer keeps the first call's contents), refuses a handle without its sub-branch arena, and
refuses a count whose task list exceeds the fixed buffer."""
import json
import os

import pytest

import graphgen
import oracle
from graphgen import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ebb():
    import torch
    import paper_2311_13798_amd as ebb
    torch.cuda.set_device(0)
    return ebb


def test_noalloc_equals_count_on_two_calls_second_smaller(ebb):
    big = ebb.Graph.from_csr(configs.rmat_scale(14))
    gs = graphgen.er_planted(400, 0.06, 2, 14, 20, seed=7)
    small = ebb.Graph.from_csr(gs)
    for G in (big, small):
        G.count(4)  # builds the sub-branch arena
    for rep in range(2):
        for G, k in ((big, 7), (small, 5)):
            print(f"case noalloc rep={rep} n={G.info.n} k={k}", flush=True)
            got = ebb.ebbkc_count_noalloc(G.handle, k)
            assert got == ebb.ebbkc_count(G.handle, k), (G.info.n, k)
    assert ebb.ebbkc_count_noalloc(small.handle, 6) == oracle.count(gs, 6)
    for k in (1, 2, 3, 4):
        assert ebb.ebbkc_count_noalloc(small.handle, k) == oracle.count(gs, k)
    big.close()
    small.close()


def test_noalloc_needs_the_arena(ebb):
    G = ebb.Graph.from_csr(graphgen.er_planted(300, 0.05, 1, 12, 12, seed=3))
    with pytest.raises(ebb.EbbkcError) as ei:
        ebb.ebbkc_count_noalloc(G.handle, 5)
    assert ei.value.status == ebb.E_INVALID_ARG
    G.count(5)
    assert ebb.ebbkc_count_noalloc(G.handle, 5) == G.count(5)
    G.close()


def test_noalloc_limit_on_the_rmat18_workload(ebb):
    # k = 5 fits the fixed buffer and equals the oracle's stored count; k = 7 needs a task list
    # larger than it (about 9e6 tasks at 40 bytes each) and is refused, after which the buffer still
    # serves a smaller count
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rmat18.json")))
    g = configs.rmat18()
    assert g.sha256() == fx["sha256"]
    G = ebb.Graph.from_csr(g)
    G.count(4)
    print("case noalloc rmat18 k=5", flush=True)
    assert ebb.ebbkc_count_noalloc(G.handle, 5) == fx["counts"]["5"]
    print("case noalloc rmat18 k=7", flush=True)
    with pytest.raises(ebb.EbbkcError) as ei:
        ebb.ebbkc_count_noalloc(G.handle, 7)
    assert ei.value.status == ebb.E_SCRATCH
    assert ebb.ebbkc_count_noalloc(G.handle, 3) == fx["counts"]["3"]
    G.close()
