"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

Usage:  python tests/golden/make_golden.py [--with-k7] [--with-k12] [--only NAME]
Every value written here comes from ``oracle`` applied to the seeded inputs of ``graphgen``.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from graphgen import configs  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def arr_sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.int32).tobytes()).hexdigest()


def graph_record(g, ks, list_ks=(), sample_ks=(), nsample=0, seed=0):
    rec = {"name": g.name, "sha256": g.sha256(), "n": g.n, "m": g.m, "max_degree": int(g.degrees().max(initial=0))}
    t0 = time.time()
    tr = oracle.truss_levelsync(g)
    rec["tau"] = tr["tau"]
    rec["rounds"] = tr["rounds"]
    rec["rank_sha256"] = arr_sha(tr["rank"])
    rec["level_sha256"] = arr_sha(tr["level"])
    rec["support_sha256"] = arr_sha(oracle.edge_support(g))
    sub = oracle.seed_sizes(g, tr["rank"])
    rec["subsize_sha256"] = arr_sha(sub)
    rec["delta"] = oracle.degeneracy(g)[1]
    rec["counts"] = {}
    for k in ks:
        t = time.time()
        rec["counts"][str(k)] = oracle.count(g, k)
        print(g.name, "k", k, rec["counts"][str(k)], f"{time.time() - t:.1f}s", flush=True)
    rec["listings"] = {}
    for k in list_ks:
        c, ho, hu, _ = oracle.list_lex(g, k, want_tuples=False)
        rec["listings"][str(k)] = {"count": c, "ordered": str(ho), "unordered": str(hu)}
    rec["seed_samples"] = {}
    if nsample:
        rng = np.random.default_rng(seed)
        lev = tr["level"]
        for k, cap in sample_ks:
            cand = np.nonzero((lev >= k - 2) & (sub >= k - 2) & (sub <= cap))[0]
            pick = rng.choice(cand, size=min(nsample, cand.size), replace=False) if cand.size else cand
            cnt = oracle.seed_counts(g, tr["rank"], k, pick)
            rec["seed_samples"][str(k)] = {"eids": pick.tolist(), "counts": [str(int(x)) for x in cnt]}
    rec["oracle_seconds"] = round(time.time() - t0, 1)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--with-k7", action="store_true")
    ap.add_argument("--with-k12", action="store_true")
    ap.add_argument("--only", default="")
    args = ap.parse_args()
    if args.only in ("", "er_small"):
        g = configs.er_small()
        rec = graph_record(g, ks=range(1, 8), list_ks=(3, 4))
        json.dump(rec, open(os.path.join(OUT, "er_small.json"), "w"), indent=1)
    if args.only in ("", "rmat18"):
        g = configs.rmat18()
        ks = [1, 2, 3, 4, 5, 6] + ([7] if args.with_k7 else [])
        rec = graph_record(g, ks=ks, sample_ks=((5, 1000), (7, 100), (9, 70)), nsample=300, seed=1)
        json.dump(rec, open(os.path.join(OUT, "rmat18.json"), "w"), indent=1)
    if args.only in ("", "rmat18_list5"):
        # the full k = 5 listing of R-MAT s18 (5.5e10 tuples): count and order-independent checksum
        g = configs.rmat18()
        t = time.time()
        c, ho, hu, _ = oracle.list_lex(g, 5, want_tuples=False)
        rec = {"name": g.name, "sha256": g.sha256(), "k": 5, "count": c, "unordered": str(hu),
               "ordered": str(ho), "oracle_seconds": round(time.time() - t, 1)}
        print("rmat18 list k=5", c, hu, f"{time.time() - t:.1f}s", flush=True)
        json.dump(rec, open(os.path.join(OUT, "rmat18_list5.json"), "w"), indent=1)
    if args.only in ("", "cl1m"):
        # Chung-Lu n = 10^6 with 200 planted cliques (the dense-branch early-termination workload)
        g = configs.cl_planted()
        ks = [1, 2, 3, 4, 5, 8, 10] + ([12] if args.with_k12 else [])
        rec = graph_record(g, ks=ks, sample_ks=((8, 200), (10, 200), (12, 200)), nsample=300, seed=3)
        json.dump(rec, open(os.path.join(OUT, "cl1m.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
