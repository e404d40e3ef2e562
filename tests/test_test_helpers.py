"""The expected-value helpers of the GPU tests, pinned on the CPU: the independence polynomial of a
union of paths and cycles (3-plex tests) equals the oracle's clique counts of the complement graph and
brute force; the sequential greedy colouring is proper and greedy; the level-synchronous core peel
orders every vertex with at most delta later neighbours and equals a pure-Python peel."""
import importlib.util
import itertools
import os
import random

import numpy as np

import graphgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _load(name):
    spec = importlib.util.spec_from_file_location(name, os.path.join(HERE, name + ".py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


tplex = _load("test_gpu_tplex")
orderings = _load("test_gpu_orderings")


def test_independence_polynomial_against_oracle_and_brute_force():
    for seed in range(12):
        n = 6 + seed % 9
        g, missing = tplex.complement_of_paths_and_cycles(n, seed)
        poly = tplex.independence_poly(n, missing)
        ms = {tuple(e) for e in missing}
        for l in range(1, n + 2):
            want = poly[l] if l < len(poly) else 0
            assert oracle.count(g, l) == want, (seed, l)
            if n <= 12:
                brute = sum(1 for s in itertools.combinations(range(n), l)
                            if not any((a, b) in ms for a, b in itertools.combinations(s, 2)))
                assert brute == want, (seed, l)
    # every vertex of the complement misses at most two others (a 3-plex)
    g, missing = tplex.complement_of_paths_and_cycles(200, 7)
    deg = np.bincount(np.array(missing).ravel(), minlength=200)
    assert deg.max() <= 2


def test_greedy_colouring_helper():
    rng = random.Random(1)
    for seed in range(6):
        g = graphgen.er(rng.randint(20, 120), rng.uniform(0.05, 0.5), seed)
        col = orderings.greedy_colouring(g)
        eu, ev = oracle.edge_list(g)
        assert (col[eu] != col[ev]).all()
        # greedy: each vertex's colour is the least not used by its neighbours visited before it
        deg = np.diff(g.row_ptr)
        order = sorted(range(g.n), key=lambda v: (-deg[v], v))
        pos = np.empty(g.n, np.int64)
        pos[order] = np.arange(g.n)
        for v in range(g.n):
            nb = g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]
            used = {int(col[w]) for w in nb if pos[w] < pos[v]}
            assert int(col[v]) == min(c for c in range(1, len(used) + 2) if c not in used)


def test_core_peel_helper():
    for seed in range(6):
        g = graphgen.rmat(8, 8, seed=seed + 1)
        pos = orderings.core_peel_order(g)
        assert np.array_equal(np.sort(pos), np.arange(g.n))
        _, delta = oracle.degeneracy(g)
        assert orderings.out_degrees(g, pos).max() <= delta
        # pure-Python level-synchronous peel
        adj = [set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]
        alive, deg, placed, s, want = set(range(g.n)), [len(a) for a in adj], 0, 0, [0] * g.n
        while alive:
            front = sorted(v for v in alive if deg[v] <= s)
            if not front:
                s = min(deg[v] for v in alive)
                continue
            for i, v in enumerate(front):
                want[v] = placed + i
            placed += len(front)
            alive -= set(front)
            for v in front:
                for w in adj[v]:
                    if w in alive:
                        deg[w] -= 1
        assert list(pos) == want
