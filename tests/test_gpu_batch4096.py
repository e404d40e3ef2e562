"""The batched workload at its stated size: 4,096 Erdos-Renyi graphs, n U{50..5000}, p U[0.005, 0.2],
20 % with one planted clique of U{20..40}, k U{3..10} per graph, about 1.8e9 edges in all.  Every graph
is prepared and resident in device memory, the whole batch runs as one fused launch per width class
(each task building its sub-branch in LDS: the graphs' arenas would need about 700 GB) and is replayed
from its HIP graph, and every per-graph count equals the oracle's stored count
(tests/golden/batch4096.json, written by tests/golden/make_golden.py from the oracle alone)."""
import concurrent.futures as cf
import json
import os
import time

import pytest

from graphgen import configs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch4096.json")


def generate(params, threads=16):
    # the generators are C code called through ctypes (the GIL is released), so threads overlap
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(configs.batch_graph, params))


@pytest.mark.timeout(900)
def test_batch_of_4096_graphs_at_full_size():
    import torch
    import paper_2311_13798_amd as ebb
    torch.cuda.set_device(0)
    ref = json.load(open(GOLDEN))
    assert ref["complete"]
    gold = {r["index"]: r for r in ref["graphs"]}
    params = configs.batch_params(4096)
    assert len(gold) == len(params) == 4096
    t0 = time.time()
    Gs, ks = [], []
    for i0 in range(0, 4096, 256):  # generate, check and prepare in groups (bounded host memory)
        part = params[i0:i0 + 256]
        for p, g in zip(part, generate(part)):
            r = gold[p["index"]]
            assert (g.n, g.m, g.sha256()) == (r["n"], r["m"], r["sha256"]), p["index"]
            Gs.append(ebb.Graph.from_csr(g))
            ks.append(int(p["k"]))
        print(f"case batch4096 prepared {len(Gs)} graphs in {time.time() - t0:.1f}s", flush=True)
    assert sum(G.info.m for G in Gs) == sum(r["m"] for r in gold.values())
    o = ebb.ebbkc_default_options()
    o.batch_build = ebb.BATCH_BUILD
    B = ebb.Batch(Gs, ks, options=o)
    print(f"case batch4096 batch created, {B.info()[0]} tasks, {time.time() - t0:.1f}s", flush=True)
    want = [int(gold[p["index"]]["count"]) for p in params]
    got = B.run(use_graph=False)
    print(f"case batch4096 eager run {B.info()[1]:.0f} ms", flush=True)
    assert got == want
    got = B.run(use_graph=True)
    print(f"case batch4096 graph replay {B.info()[1]:.0f} ms", flush=True)
    assert got == want
    B.close()
    for G in Gs:
        G.close()
