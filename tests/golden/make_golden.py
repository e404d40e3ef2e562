"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

Usage:  python tests/golden/make_golden.py [--with-k7] [--with-k12] [--only NAME] [--threads T]
Every value written here comes from ``oracle`` applied to the seeded inputs of ``graphgen``.

Targets (``--only``): er_small, rmat18, rmat18_list5, cl1m (written by the default run), and the
long ones run on their own: rmat18_k8 (the full 8-clique count of the R-MAT scale-18 workload,
hours of CPU), rmat18_w3 (per-seed counts at k = 8 and 9 of sampled seeds whose sub-branch has
129..192 vertices, the three-word bitmap class), batch4096 (the exact count of every graph of the
batched workload at its own k), served (R-MAT scale 13 at k = 3..12 for the served-form tests).
"""
import argparse
import concurrent.futures as cf
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


def rmat18_k8(threads):
    g = configs.rmat18()
    t = time.time()
    c = oracle.count(g, 8, threads=threads)
    rec = {"name": g.name, "sha256": g.sha256(), "k": 8, "count": c, "threads": threads,
           "oracle_seconds": round(time.time() - t, 1)}
    print("rmat18 k=8", c, f"{time.time() - t:.1f}s", flush=True)
    json.dump(rec, open(os.path.join(OUT, "rmat18_k8.json"), "w"), indent=1)


def rmat18_w3(threads, per_k=((8, 40), (9, 32)), lo=129, hi=192, seed=11):
    """Per-seed counts of sampled seeds of the three-word class (sub-branch of lo..hi vertices).
    The seeds are independent, so they run in a thread pool (the oracle call releases the GIL)."""
    g = configs.rmat18()
    t0 = time.time()
    tr = oracle.truss_levelsync(g)
    sub = oracle.seed_sizes(g, tr["rank"])
    rng = np.random.default_rng(seed)
    rec = {"name": g.name, "sha256": g.sha256(), "rank_sha256": arr_sha(tr["rank"]),
           "subsize_range": [lo, hi], "seed_samples": {}}
    for k, ns in per_k:
        cand = np.nonzero((tr["level"] >= k - 2) & (sub >= lo) & (sub <= hi))[0]
        pick = np.sort(rng.choice(cand, size=min(ns, cand.size), replace=False))
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            got = list(ex.map(lambda e: int(oracle.seed_counts(g, tr["rank"], k, np.array([e]))[0]), pick))
        rec["seed_samples"][str(k)] = {"eids": pick.tolist(), "subsizes": sub[pick].tolist(),
                                       "counts": [str(x) for x in got]}
        print("rmat18 w3 k", k, len(pick), "seeds", sum(got), f"{time.time() - t0:.1f}s", flush=True)
    rec["oracle_seconds"] = round(time.time() - t0, 1)
    json.dump(rec, open(os.path.join(OUT, "rmat18_w3seeds.json"), "w"), indent=1)


def _batch_one(p):
    g = configs.batch_graph(p)
    t = time.time()
    c = oracle.count(g, int(p["k"]), threads=1)
    return {"index": p["index"], "n": g.n, "m": g.m, "k": int(p["k"]), "clique": p["clique"],
            "sha256": g.sha256(), "count": c, "seconds": round(time.time() - t, 3)}


def batch4096(threads, count=4096):
    """Exact count of every graph of the batched workload at its own k, one graph per worker
    process (graphs generated, counted and dropped one at a time), in index order, so that the
    graphs finished so far are a uniform sample; the file is rewritten every 32 graphs."""
    params = configs.batch_params(count)
    t0 = time.time()
    out = {}
    path = os.path.join(OUT, "batch4096.json")

    def dump(done):
        rec = {"workload": "batched workload: graph i from seed splitmix64(1 ^ i), n U{50..5000}, "
                           "p U[0.005, 0.2], 20% with one planted clique of U{20..40}, k U{3..10}",
               "complete": done, "graphs": [out[i] for i in sorted(out)],
               "oracle_seconds": round(time.time() - t0, 1), "threads": threads}
        tmp = path + ".tmp"
        json.dump(rec, open(tmp, "w"))
        os.replace(tmp, path)

    with cf.ProcessPoolExecutor(max_workers=threads) as ex:
        for i, r in enumerate(ex.map(_batch_one, params, chunksize=1)):
            out[r["index"]] = r
            if i % 32 == 31:
                dump(False)
                print("batch4096", i + 1, f"{time.time() - t0:.1f}s", flush=True)
    dump(True)


def served():
    """Oracle counts of the served-form test catalogue graphs too large to count inside a test."""
    rec = {"graphs": {}}
    for name, g, ks in (("rmat13", configs.rmat_scale(13), range(3, 13)),):
        t = time.time()
        counts = {str(k): oracle.count(g, k) for k in ks}
        rec["graphs"][name] = {"sha256": g.sha256(), "n": g.n, "m": g.m, "counts": counts,
                               "oracle_seconds": round(time.time() - t, 1)}
        print("served", name, counts, flush=True)
    json.dump(rec, open(os.path.join(OUT, "served.json"), "w"), indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--with-k7", action="store_true")
    ap.add_argument("--with-k12", action="store_true")
    ap.add_argument("--only", default="")
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    th = args.threads or oracle.default_threads()
    if args.only == "rmat18_k8":
        return rmat18_k8(th)
    if args.only == "rmat18_w3":
        return rmat18_w3(th)
    if args.only == "batch4096":
        return batch4096(th)
    if args.only == "served":
        return served()
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
