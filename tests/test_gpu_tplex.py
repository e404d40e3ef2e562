"""t-plex early termination (every vertex misses at most t - 1 others; Section 5, Algorithm kCtPlex).
t = 3: graphs whose missing pairs form disjoint paths and cycles, counted with t = 1, 2, 3 and the
paper's rule (t = 3 when k > tau / 2); t = 4, 5: graphs whose missing pairs have maximum degree t - 1,
counted by kCtPlex's branching on the inverse graph, and general graphs against the oracle.  The expected N_k is the coefficient of x^k in the independence
polynomial of the missing-pair graph, computed here by plain vertex deletion
(I(H) = I(H - v) + x I(H - N[v])) with Python integers, and by the oracle where it is fast."""
import functools
import random

import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def independence_poly(n, edges):
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)

    @functools.lru_cache(maxsize=None)
    def ip(vs):
        if not vs:
            return (1,)
        v = min(vs, key=lambda u: (-len(adj[u] & vs), u))
        if not (adj[v] & vs):  # isolated: factor (1 + x)
            rest = ip(vs - {v})
            return tuple((rest[i] if i < len(rest) else 0) + (rest[i - 1] if i >= 1 else 0)
                         for i in range(len(rest) + 1))
        a, b = ip(vs - {v}), ip(vs - {v} - adj[v])
        out = [0] * max(len(a), len(b) + 1)
        for i, c in enumerate(a):
            out[i] += c
        for i, c in enumerate(b):
            out[i + 1] += c
        return tuple(out)

    # components separately
    seen, poly = set(), [1]
    for s in range(n):
        if s in seen:
            continue
        comp, stack = set(), [s]
        while stack:
            u = stack.pop()
            if u in comp:
                continue
            comp.add(u)
            stack.extend(adj[u] - comp)
        seen |= comp
        p = ip(frozenset(comp))
        new = [0] * (len(poly) + len(p) - 1)
        for i, x in enumerate(poly):
            for j, y in enumerate(p):
                new[i + j] += x * y
        poly = new
    return poly


def complement_of_paths_and_cycles(n, seed):
    rng = random.Random(seed)
    perm = list(range(n))
    rng.shuffle(perm)
    missing, i = [], 0
    while i < n:
        L = rng.choice([1, 1, 2, 2, 3, 4, 5, 7, 9, 13])
        comp = perm[i:i + L]
        i += L
        for a, b in zip(comp, comp[1:]):
            missing.append((min(a, b), max(a, b)))
        if len(comp) >= 3 and rng.random() < 0.4:
            missing.append((min(comp[0], comp[-1]), max(comp[0], comp[-1])))
    ms = set(missing)
    edges = [[a, b] for a in range(n) for b in range(a + 1, n) if (a, b) not in ms]
    return graphgen.from_edges(n, edges), missing


@pytest.fixture(scope="module")
def ebb():
    import torch
    import paper_2311_13798_amd as m
    torch.cuda.set_device(0)
    m.load_library()
    return m


@pytest.mark.parametrize("n,seed", [(20, 1), (40, 2), (63, 3), (90, 4), (150, 5), (230, 6)])
def test_three_plex_counts(ebb, n, seed):
    g, missing = complement_of_paths_and_cycles(n, seed)
    poly = independence_poly(n, missing)
    ks = sorted({3, 4, 5, 6, 8, n // 3, n // 2 - 1, n // 2, n // 2 + 1, len(poly) - 2, len(poly) - 1, len(poly)})
    for t in (0, 1, 2, 3):
        o = ebb.ebbkc_default_options()
        o.t_plex = t
        G = ebb.Graph.from_csr(g, options=o)
        tau = G.info.tau
        for k in ks:
            if k < 3:
                continue
            want = poly[k] if k < len(poly) else 0
            three = t == 3 or (t == 0 and 2 * k > tau)
            if want >= 1 << 128 or (not three and k > 6):
                continue  # branching without the 3-plex form would take too long
            print(f"case 3-plex n={n} t={t} k={k}", flush=True)
            assert G.count128(k) == want, (n, t, k)
        G.close()


def test_three_plex_counts_match_the_oracle(ebb):
    for seed in range(6):
        g, missing = complement_of_paths_and_cycles(28, 100 + seed)
        G = ebb.Graph.from_csr(g)
        o3 = ebb.ebbkc_default_options()
        o3.t_plex = 3
        G3 = ebb.Graph.from_csr(g, options=o3)
        for k in range(3, 12):
            want = oracle.count(g, k)
            assert G.count(k) == want and G3.count(k) == want, (seed, k)
        G.close()
        G3.close()


def complement_of_bounded_degree(n, maxdeg, seed, tries=4):
    """A graph whose missing pairs form a random graph of maximum degree maxdeg (so the graph is a
    (maxdeg + 1)-plex), with some vertices missing nobody."""
    rng = random.Random(seed)
    deg = [0] * n
    missing = set()
    for _ in range(tries * n):
        a, b = rng.randrange(n), rng.randrange(n)
        if a == b or (min(a, b), max(a, b)) in missing or deg[a] >= maxdeg or deg[b] >= maxdeg:
            continue
        missing.add((min(a, b), max(a, b)))
        deg[a] += 1
        deg[b] += 1
    edges = [[a, b] for a in range(n) for b in range(a + 1, n) if (a, b) not in missing]
    return graphgen.from_edges(n, edges), sorted(missing)


@pytest.mark.parametrize("t,n,seed,kmax", [(4, 24, 1, 24), (5, 24, 2, 24), (4, 40, 3, 10), (5, 40, 4, 10),
                                          (4, 64, 5, 7), (5, 64, 6, 7)])
def test_t_plex_counts_by_inverse_graph_branching(ebb, t, n, seed, kmax):
    # t = 4, 5: Algorithm kCtPlex (branching on the inverse graph, the vertices adjacent to all others
    # in closed form) on graphs that are t-plexes but not 3-plexes; N_k is the independence
    # polynomial of the missing pairs (the oracle's count for n = 64)
    g, missing = complement_of_bounded_degree(n, t - 1, seed)
    degs = [0] * n
    for a, b in missing:
        degs[a] += 1
        degs[b] += 1
    assert max(degs) == t - 1
    poly = independence_poly(n, missing) if n <= 40 else None
    o = ebb.ebbkc_default_options()
    o.t_plex = t
    G = ebb.Graph.from_csr(g, options=o)
    for k in range(3, kmax + 1):
        if poly is not None:
            want = poly[k] if k < len(poly) else 0
        else:
            want = oracle.count(g, k)
        print(f"case t-plex t={t} n={n} k={k}", flush=True)
        assert G.count128(k) == want, (t, n, k)
    G.close()


@pytest.mark.parametrize("t", [4, 5])
def test_t_plex_counts_match_the_oracle_on_general_graphs(ebb, t):
    # graphs where only some candidate sets are t-plexes: planted dense parts in sparse noise, and
    # near-cliques; every t gives the oracle's counts
    gs = [graphgen.er_planted(300, 0.04, 3, 18, 26, seed=40 + t), complement_of_bounded_degree(36, t, 7 + t)[0],
          graphgen.er(90, 0.6, seed=t)]
    for g in gs:
        o = ebb.ebbkc_default_options()
        o.t_plex = t
        G = ebb.Graph.from_csr(g, options=o)
        for k in range(3, 11):
            print(f"case t-plex general t={t} n={g.n} k={k}", flush=True)
            assert G.count(k) == oracle.count(g, k), (t, g.n, k)
        G.close()
