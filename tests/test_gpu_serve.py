"""Served form: every request's count equals the standalone count of the same (graph, k), whatever
requests shared its epoch; a small budget forces many epochs, a large one merges requests."""
import numpy as np
import pytest

import graphgen
from graphgen import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def catalogue():
    import torch
    import paper_2311_13798_amd as ebb
    torch.cuda.set_device(0)
    gs = [configs.er_small(), graphgen.rmat(10, 16, seed=1), graphgen.er_planted(300, 0.05, 1, 25, 25, 2),
          graphgen.cocktail_party(10), configs.cl_planted(10000, nplant=2), graphgen.empty(5)]
    Gs = [ebb.Graph.from_csr(g) for g in gs]
    alone = {(i, k): G.count(k) for i, G in enumerate(Gs) for k in range(1, 13)}
    yield ebb, Gs, alone
    for G in Gs:
        G.close()


@pytest.mark.parametrize("budget", [1 << 20, 1 << 40])
def test_results_equal_alone_and_in_the_mix(catalogue, budget):
    from paper_2311_13798_amd.serve import Server, poisson_requests
    ebb, Gs, alone = catalogue
    S = Server(Gs, budget)
    reqs = poisson_requests(rate=2000.0, count=300, n_graphs=len(Gs), k_lo=1, k_hi=12, seed=budget % 97)
    res = S.run_stream(reqs)
    for (off, g, k), r in zip(reqs, res):
        assert r["status"] == 0 and r["graph"] == g and r["k"] == k
        assert r["count"] == alone[(g, k)], (g, k)
        assert r["done_ms"] >= r["admit_ms"] >= r["arrival_ms"]
    st = S.stats()
    assert st["submitted"] == len(reqs) and st["outstanding"] == 0
    if budget == 1 << 40:
        assert st["max_epoch_requests"] > 1  # requests that arrived together shared a launch
    S.close()


def test_burst_then_drain(catalogue):
    from paper_2311_13798_amd.serve import Server
    ebb, Gs, alone = catalogue
    S = Server(Gs, 1 << 40)
    rng = np.random.default_rng(5)
    pairs = [(int(rng.integers(0, len(Gs))), int(rng.integers(3, 10))) for _ in range(200)]
    ids = [S.submit(g, k) for g, k in pairs]
    got = {}
    while len(got) < len(ids):
        for r in S.poll(wait=True):
            got[r["id"]] = r
    for i, (g, k) in zip(ids, pairs):
        assert got[i]["count"] == alone[(g, k)]
    S.close()


def test_light_requests_run_beside_a_heavy_one():
    # R-MAT scale 13 at k = 12 takes ~2.3 s alone; requests arriving while it runs start in other
    # epoch slots and finish long before it, each with its standalone count
    import time

    import torch
    import paper_2311_13798_amd as ebb
    from paper_2311_13798_amd.serve import Server
    torch.cuda.set_device(0)
    heavy = ebb.Graph.from_csr(configs.rmat_scale(13))
    lights = [ebb.Graph.from_csr(g) for g in (configs.er_small(), graphgen.rmat(10, 16, seed=1),
                                              graphgen.er_planted(300, 0.05, 1, 25, 25, 2))]
    want_heavy = heavy.count(12)
    alone = {(i, k): G.count(k) for i, G in enumerate(lights) for k in range(3, 8)}
    S = Server([heavy] + lights, 1 << 40)
    hid = S.submit(0, 12)
    time.sleep(0.05)
    ids = {}
    for i in range(45):
        g, k = i % len(lights), 3 + (i // len(lights)) % 5
        ids[S.submit(1 + g, k)] = (g, k)
        time.sleep(0.002)
    res = {}
    while len(res) < len(ids) + 1:
        for r in S.poll(wait=True):
            res[r["id"]] = r
    S.close()
    assert res[hid]["count"] == want_heavy
    for i, gk in ids.items():
        assert res[i]["status"] == 0 and res[i]["count"] == alone[gk]
    before = sum(1 for i in ids if res[i]["done_ms"] < res[hid]["done_ms"])
    assert before >= 40, before
    for G in [heavy] + lights:
        G.close()
