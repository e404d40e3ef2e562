"""Listing parity (HIP path through the C-ABI vs the CPU oracle): byte-identical sorted buffers,
identical checksums, set equality of unsorted buffers, rank-range chunks, buffer-too-small."""
import json
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


def gpu_list(ebb, G, k, sorted_=True, r_begin=0, r_end=-1, cap=None):
    import torch
    n = G.count(k) if (r_begin == 0 and r_end == -1) else G.count_range(k, r_begin, r_end if r_end >= 0 else G.info.m) if k >= 3 else None
    if cap is None:
        cap = max(int(n or 1), 1) if n is not None else 1 << 20
    buf = torch.zeros((max(cap, 1), k), dtype=torch.int32, device="cuda")
    w, ho, hu = ebb.ebbkc_list(G.handle, k, buf, cap, ebb.LIST_SORTED if sorted_ else 0, r_begin, r_end)
    return w, ho, hu, buf[:w].cpu().numpy()


def graphs():
    return [
        ("appendix_b", graphgen.from_edges(4, json.load(open(os.path.join(GOLDEN, "appendix_b.json")))["edges"])),
        ("er_small", configs.er_small()),
        ("er_planted", graphgen.er_planted(300, 0.06, 2, 12, 18, 5)),
        ("cocktail8", graphgen.cocktail_party(8)),
        ("K10", graphgen.complete(10)),
        ("rmat10", graphgen.rmat(10, 16, seed=3)),
    ]


@pytest.mark.parametrize("name,g", graphs(), ids=lambda x: x if isinstance(x, str) else "")
def test_sorted_listing_matches_oracle(ebb, name, g):
    G = ebb.Graph.from_csr(g)
    for k in range(1, 8):
        c, ho, hu, ref = oracle.list_lex(g, k)
        if c > 2_000_000:
            continue
        print(f"case list {name} k={k} n={c}", flush=True)
        w, gho, ghu, tup = gpu_list(ebb, G, k)
        assert w == c
        assert (gho, ghu) == (ho, hu), (name, k)
        assert np.array_equal(tup, ref), (name, k)
    G.close()


def test_unsorted_listing_is_the_same_set(ebb):
    g = graphgen.er_planted(400, 0.05, 2, 14, 20, 11)
    G = ebb.Graph.from_csr(g)
    for k in (3, 4, 5, 6, 7):
        c, ho, hu, ref = oracle.list_lex(g, k)
        w, gho, ghu, tup = gpu_list(ebb, G, k, sorted_=False)
        assert w == c and ghu == hu
        assert (np.diff(tup, axis=1) > 0).all()  # ascending inside each tuple
        got = tup[np.lexsort(tup.T[::-1])]
        assert np.array_equal(got, ref)
    G.close()


def test_rank_range_chunks_concatenate_to_the_listing(ebb):
    g = graphgen.rmat(11, 16, seed=7)
    G = ebb.Graph.from_csr(g)
    m = G.info.m
    cuts = [0, m // 5, m // 2, (3 * m) // 4, m]
    for k in (3, 5, 6):
        c, ho, hu, ref = oracle.list_lex(g, k)
        parts = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            cap = max(G.count_range(k, a, b), 1)
            w, _, _, tup = gpu_list(ebb, G, k, sorted_=False, r_begin=a, r_end=b, cap=cap)
            parts.append(tup)
        allt = np.concatenate(parts)
        assert allt.shape[0] == c
        assert np.array_equal(allt[np.lexsort(allt.T[::-1])], ref)
    G.close()


def test_buffer_too_small_reports_the_count(ebb):
    import torch
    g = configs.er_small()
    G = ebb.Graph.from_csr(g)
    buf = torch.zeros((10, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(ebb.EbbkcError) as ei:
        ebb.ebbkc_list(G.handle, 3, buf, 10)
    assert ei.value.status == ebb.E_BUFFER_TOO_SMALL
    assert str(oracle.count(g, 3)) in str(ei.value)
    G.close()


def test_listing_of_a_split_heavy_seed(ebb):
    # a planted 40-clique: its root sub-branches are split into per-vertex tasks
    g = graphgen.er_planted(200, 0.02, 1, 40, 40, 3)
    o = ebb.ebbkc_default_options()
    o.split_threshold = 1000
    G = ebb.Graph.from_csr(g, options=o)
    for k in (6, 7, 8):
        c, ho, hu, ref = oracle.list_lex(g, k)
        assert G.count(k) == c
        w, gho, ghu, tup = gpu_list(ebb, G, k)
        assert w == c and (gho, ghu) == (ho, hu)
    G.close()


def test_er_small_listing_golden(ebb):
    fx = json.load(open(os.path.join(GOLDEN, "er_small.json")))
    g = configs.er_small()
    G = ebb.Graph.from_csr(g)
    for k, rec in fx["listings"].items():
        w, ho, hu, _ = gpu_list(ebb, G, int(k))
        assert w == rec["count"] and str(ho) == rec["ordered"] and str(hu) == rec["unordered"]
    G.close()


def test_count_seeds_match_oracle(ebb):
    g = graphgen.rmat(11, 16, seed=2)
    G = ebb.Graph.from_csr(g)
    tr = oracle.truss_levelsync(g)
    rng = np.random.default_rng(0)
    eids = rng.choice(g.m, size=300, replace=False).astype(np.int64)
    for k in (3, 4, 5, 7):
        out = np.zeros(len(eids), np.uint64)
        ebb.ebbkc_count_seeds(G.handle, k, eids, out)
        want = oracle.seed_counts(g, tr["rank"], k, eids)
        assert np.array_equal(out, want), k
    G.close()


def test_chunked_listing_equals_the_whole_listing(ebb):
    import torch
    from paper_2311_13798_amd.listing import list_in_chunks, plan_chunks
    g = graphgen.rmat(11, 16, seed=5)
    G = ebb.Graph.from_csr(g)
    for k in (4, 5, 6):
        c, ho, hu, ref = oracle.list_lex(g, k)
        cap = max(c // 7, 1)
        cuts, sizes = plan_chunks(G, k, cap)
        assert sum(sizes) == c and all(0 <= s_ <= cap for s_ in sizes)
        buf = torch.zeros((cap, k), dtype=torch.int32, device="cuda")
        parts = []
        total, ghu, nch = list_in_chunks(G, k, buf, cap, cuts=cuts,
                                         on_chunk=lambda a, b, w: parts.append(buf[:w].cpu().numpy().copy()))
        allt = np.concatenate(parts)
        assert total == c and ghu == hu and nch == len(sizes)
        assert np.array_equal(allt[np.lexsort(allt.T[::-1])], ref)
    G.close()


def test_deep_listing_of_two_overlapping_cliques(ebb):
    # two K_35 sharing 30 vertices: a seed in the shared part has 38 candidates with 25 missing pairs
    # (not a t-plex for t <= 3), so counts and listings at k = 31..36 branch deeper than the frames
    # kept in LDS and use the device-memory frames.  N_k = 2 C(35, k) - C(30, k).
    import itertools
    from math import comb
    A, B = range(0, 35), range(5, 40)
    edges = sorted({(a, b) for S in (A, B) for a, b in itertools.combinations(S, 2)})
    g = graphgen.from_edges(40, edges)
    G = ebb.Graph.from_csr(g)
    for k in (31, 33, 34, 35, 36):
        want = 2 * comb(35, k) - comb(30, k)
        print(f"case deep list k={k} n={want}", flush=True)
        assert G.count(k) == want == oracle.count(g, k)
        c, ho, hu, ref = oracle.list_lex(g, k)
        w, gho, ghu, tup = gpu_list(ebb, G, k)
        assert w == c == want
        assert (gho, ghu) == (ho, hu)
        assert np.array_equal(tup, ref)
    G.close()
