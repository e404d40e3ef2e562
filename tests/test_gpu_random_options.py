"""Seeded random cases across the option space: random graphs (sparse ER, dense ER, ER with planted
cliques, R-MAT) counted under a random combination of ordering (H, C, edge- and node-parallel VBBkC,
T), t, Rules (1) / (2), early termination, dense 4-clique weight and split threshold, at k from 3 to
one past the maximum clique size, every count against the oracle; and a few listings by checksum."""
import random

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def random_graph(rng: random.Random):
    kind = rng.choice(["sparse", "dense", "planted", "rmat"])
    seed = rng.randrange(1 << 30)
    if kind == "sparse":
        return kind, graphgen.er(rng.randint(30, 400), rng.uniform(0.02, 0.12), seed)
    if kind == "dense":
        return kind, graphgen.er(rng.randint(12, 48), rng.uniform(0.5, 0.92), seed)
    if kind == "planted":
        c = rng.randint(8, 30)
        return kind, graphgen.er_planted(rng.randint(60, 250), rng.uniform(0.02, 0.08), rng.randint(1, 3), c, c, seed)
    return kind, graphgen.rmat(rng.randint(7, 10), rng.choice([4, 8, 16]), seed=seed)


def random_options(ebb, rng: random.Random):
    o = ebb.ebbkc_default_options()
    o.ordering = rng.choice([0, 0, 1, 2, 3, 4])
    o.t_plex = rng.choice([0, 1, 2, 3])
    o.rule1 = rng.choice([0, 1])
    o.rule2 = rng.choice([0, 1])
    o.early_termination = rng.choice([0, 1, 1])
    o.dense_k4 = rng.choice([0, -1, 30, 300])
    o.split_threshold = rng.choice([0, 0, 16, 256, -1])
    return o


@pytest.fixture(scope="module")
def ebb():
    import torch
    import paper_2311_13798_amd as m
    torch.cuda.set_device(0)
    m.load_library()
    return m


@pytest.mark.parametrize("seed", range(60))
def test_random_option_combinations(ebb, seed):
    rng = random.Random(1000 + seed)
    kind, g = random_graph(rng)
    for rep in range(3):
        o = random_options(ebb, rng)
        G = ebb.Graph.from_csr(g, options=o)
        omega = G.max_clique_size()
        ks = sorted({3, 4, 5, rng.randint(3, max(3, omega)), omega, omega + 1})
        for k in ks:
            if k < 3:
                continue
            if not o.early_termination and o.ordering == 3 and k > 8:
                continue  # EBBkC-T without terminations branches through every large clique
            desc = (f"seed={seed} {kind} n={g.n} m={g.m} rep={rep} ordering={o.ordering} t={o.t_plex} "
                    f"r1={o.rule1} r2={o.rule2} et={o.early_termination} k4={o.dense_k4} "
                    f"split={o.split_threshold} k={k}")
            print("case", desc, flush=True)
            assert G.count128(k) == oracle.count(g, k), desc
        G.close()


@pytest.mark.parametrize("seed", range(8))
def test_random_listings(ebb, seed):
    import torch
    rng = random.Random(2000 + seed)
    kind, g = random_graph(rng)
    o = random_options(ebb, rng)
    G = ebb.Graph.from_csr(g, options=o)
    for k in (3, 4, 5, 6):
        c, ho, hu, _ = oracle.list_lex(g, k, want_tuples=False)
        buf = torch.empty((max(c, 1), k), dtype=torch.int32, device="cuda")
        for flags in (0, ebb.LIST_SORTED):
            w, go, gu = ebb.ebbkc_list(G.handle, k, buf, max(c, 1), flags=flags)
            assert (w, gu) == (c, hu), (seed, kind, k, flags)
            if flags:
                assert go == ho, (seed, kind, k)
                got = buf[:c].cpu().numpy()
                assert (np.diff(got, axis=1) > 0).all()
    G.close()


@pytest.mark.parametrize("seed", range(6))
def test_random_batches_and_rank_partitions(ebb, seed):
    # graphs prepared under random options, counted together in one fused batch (replayed from the
    # HIP graph twice) and alone over a random partition of the rank range; all equal the oracle
    rng = random.Random(3000 + seed)
    gs, Gs, ks = [], [], []
    for _ in range(rng.randint(3, 8)):
        kind, g = random_graph(rng)
        o = random_options(ebb, rng)
        G = ebb.Graph.from_csr(g, options=o)
        k = rng.randint(3, max(3, G.max_clique_size()))
        gs.append(g)
        Gs.append(G)
        ks.append(k)
    want = [oracle.count(g, k) for g, k in zip(gs, ks)]
    B = ebb.Batch(Gs, ks)
    for rep in range(2):
        assert list(B.run(use_graph=True)) == want, (seed, rep)
    B.close()
    for g, G, k, w in zip(gs, Gs, ks, want):
        cuts = sorted({0, g.m, *[rng.randint(0, g.m) for _ in range(3)]})
        assert sum(G.count_range(k, a, b) for a, b in zip(cuts, cuts[1:])) == w, (seed, k)
        G.close()
