"""The synthetic workloads, by name and size.

The paper evaluates on real graphs from a public network repository (Section 6.1, Table 1) that
are not available here; these seeded graphs stand in for them, with the sizes, degree skew and
dense planted structure described next to each one.
"""
from __future__ import annotations

import numpy as np

from . import Graph, chung_lu, er, er_planted, rmat, splitmix64

# (1) small plain workload: Erdos-Renyi G(2000, 0.01), seed 1, k = 4 count + listing checksum.
ER_SMALL = dict(n=2000, p=0.01, seed=1)
# (2) headline workload: R-MAT scale 18, edge factor 16, (a,b,c,d) = (0.57,0.19,0.19,0.05),
#     symmetrised, deduplicated, loops dropped; counts at k = 5, 7, 9, listing at k = 5.
RMAT18 = dict(scale=18, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=1)
RMAT18_KS = (5, 7, 9)
# (3) dense-branch stress: Chung-Lu n = 10^6, exponent 2.1, mean degree 30, 200 planted
#     cliques of size uniform 30..60; counts at k = 8, 10, 12.
CL_PLANTED = dict(n=1_000_000, gamma=2.1, mean_deg=30.0, nplant=200, smin=30, smax=60, seed=1)
CL_KS = (8, 10, 12)


def er_small() -> Graph:
    return er(**ER_SMALL)


def rmat18() -> Graph:
    return rmat(**RMAT18)


def rmat_scale(scale: int, seed: int = 1) -> Graph:
    return rmat(scale, 16, 0.57, 0.19, 0.19, seed)


def cl_planted(n: int = CL_PLANTED["n"], nplant: int | None = None, seed: int = 1) -> Graph:
    if nplant is None:
        nplant = max(2, (200 * n) // 1_000_000)
    return chung_lu(n, CL_PLANTED["gamma"], CL_PLANTED["mean_deg"], nplant,
                    CL_PLANTED["smin"], CL_PLANTED["smax"], seed)


def batch_params(count: int = 4096, seed: int = 1):
    """Parameters of the batched workload's graphs: graph i draws from seed splitmix64(seed ^ i):
    n ~ U{50..5000}, p ~ U[0.005, 0.2], k ~ U{3..10}; exactly floor(0.2*count) graphs (a seeded
    choice) carry one planted clique of size U{20..40}."""
    out = []
    rs = np.random.Generator(np.random.PCG64(seed))
    planted = set(rs.choice(count, size=int(0.2 * count), replace=False).tolist())
    for i in range(count):
        s = splitmix64(seed ^ i)
        r = np.random.Generator(np.random.PCG64(s))
        n = int(r.integers(50, 5001))
        p = float(r.uniform(0.005, 0.2))
        k = int(r.integers(3, 11))
        size = int(r.integers(20, 41)) if i in planted else 0
        out.append(dict(index=i, n=n, p=p, k=k, clique=size, seed=s))
    return out


def batch_graph(params) -> Graph:
    nplant = 1 if params["clique"] else 0
    size = max(2, min(params["clique"], params["n"])) if nplant else 2
    g = er_planted(params["n"], params["p"], nplant, size, size, params["seed"])
    g.name = f"batch{params['index']}"
    return g
