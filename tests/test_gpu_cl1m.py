"""The dense-branch workload at full size (Chung-Lu n = 10^6, exponent 2.1, mean degree 30, 200
planted cliques of 30..60, seed 1) against stored oracle values (tests/golden/cl1m.json, written by
tests/golden/make_golden.py from the oracle alone): per-edge arrays by SHA-256, counts at
k = 1..5, 8, 10, 12 bit-exact, and per-seed counts at k = 8, 10, 12 on 300 sampled seeds each."""
import hashlib
import json
import os

import numpy as np
import pytest

from graphgen import configs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cl1m.json")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_2311_13798_amd as ebb
    torch.cuda.set_device(0)
    fx = json.load(open(GOLDEN))
    g = configs.cl_planted()
    assert g.sha256() == fx["sha256"]
    G = ebb.Graph.from_csr(g)
    yield ebb, fx, g, G
    G.close()


def test_prepare_arrays(setup):
    ebb, fx, g, G = setup
    assert (G.info.n, G.info.m, G.info.tau, G.info.rounds) == (fx["n"], fx["m"], fx["tau"], fx["rounds"])
    assert sha(G.export(ebb.ARR_SUPPORT)) == fx["support_sha256"]
    assert sha(G.export(ebb.ARR_LEVEL)) == fx["level_sha256"]
    assert sha(G.export(ebb.ARR_RANK)) == fx["rank_sha256"]
    assert sha(G.export(ebb.ARR_SUBSIZE)) == fx["subsize_sha256"]


def test_counts(setup):
    ebb, fx, g, G = setup
    for k, v in fx["counts"].items():
        print(f"case cl1m count k={k}", flush=True)
        assert G.count(int(k)) == v, k


@pytest.mark.parametrize("k", [8, 10, 12])
def test_sampled_seed_counts(setup, k):
    ebb, fx, g, G = setup
    rec = fx["seed_samples"][str(k)]
    eids = np.array(rec["eids"], dtype=np.int64)
    out = np.zeros(len(eids), np.uint64)
    ebb.ebbkc_count_seeds(G.handle, k, eids, out)
    assert [int(x) for x in out] == [int(x) for x in rec["counts"]]


@pytest.mark.parametrize("name,kw,ks", [("t3", {"t_plex": 3}, (8, 10)), ("vbbkc_ep", {"ordering": 2}, (5, 8, 10)),
                                        ("vbbkc_np", {"ordering": 4}, (5, 8, 10))])
def test_counts_under_variants(setup, name, kw, ks):
    # 3-plex terminations forced on (the rule picks t = 2 here since 2k <= tau = 82) and the
    # edge- and node-parallel VBBkC roots (degeneracy order): the stored oracle counts at full size
    ebb, fx, g, _ = setup
    o = ebb.ebbkc_default_options()
    for key, v in kw.items():
        setattr(o, key, v)
    G = ebb.Graph.from_csr(g, options=o)
    for k in ks:
        print(f"case cl1m {name} k={k}", flush=True)
        assert G.count(k) == fx["counts"][str(k)], k
    G.close()
