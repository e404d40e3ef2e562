"""Served form driver: Poisson request streams against the library's continuous-batching server.

The server itself (admission, epochs, fused launches) is native code in libebbkc
(``ebbkc_server_*``); this module only generates seeded arrival times and (graph, k) choices,
submits requests at their arrival times, collects results and summarises latency.
"""
from __future__ import annotations

import time

import numpy as np

from . import (Graph, ebbkc_server_cancel, ebbkc_server_create, ebbkc_server_destroy, ebbkc_server_poll,
               ebbkc_server_stats, ebbkc_server_submit)


def poisson_requests(rate: float, count: int, n_graphs: int, k_lo: int = 3, k_hi: int = 12, seed: int = 1,
                     weights=None):
    """Arrival offsets (seconds) of a Poisson process of the given rate, and a (graph, k) per request
    drawn uniformly (graph weights optional)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    p = None if weights is None else np.asarray(weights, float) / np.sum(weights)
    graphs = rng.choice(n_graphs, size=count, p=p)
    ks = rng.integers(k_lo, k_hi + 1, size=count)
    return [(float(a), int(g), int(k)) for a, g, k in zip(t, graphs, ks)]


class Server:
    """A resident catalogue of prepared graphs served with continuous batching."""

    def __init__(self, graphs: list[Graph], budget_bytes: int, options=None):
        self._graphs = list(graphs)
        self._s = ebbkc_server_create([G.handle for G in self._graphs], budget_bytes, options)

    def submit(self, graph: int, k: int) -> int:
        return ebbkc_server_submit(self._s, graph, k)

    def cancel(self, rid: int):
        ebbkc_server_cancel(self._s, rid)

    def poll(self, wait: bool = False):
        return ebbkc_server_poll(self._s, 4096, wait)

    def stats(self):
        return dict(zip(("submitted", "epochs", "max_epoch_requests", "outstanding"), ebbkc_server_stats(self._s)))

    def run_stream(self, requests):
        """Submit each (offset_s, graph, k) at its offset; return the results in request order."""
        ids = {}
        t0 = time.perf_counter()
        out = []
        for off, g, k in requests:
            while True:
                now = time.perf_counter() - t0
                if now >= off:
                    break
                if off - now > 2e-3:
                    time.sleep(off - now - 1e-3)
            ids[self.submit(g, k)] = len(ids)
            out.extend(self.poll(wait=False))
        while len(out) < len(requests):
            out.extend(self.poll(wait=True))
        res = [None] * len(requests)
        for r in out:
            res[ids[r["id"]]] = r
        return res

    def close(self):
        if getattr(self, "_s", None):
            ebbkc_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def summarize(results):
    lat = np.array([r["done_ms"] - r["arrival_ms"] for r in results])
    start = min(r["arrival_ms"] for r in results)
    end = max(r["done_ms"] for r in results)
    total = sum(r["count"] for r in results)
    return dict(requests=len(results), p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), makespan_s=(end - start) / 1e3, kcliques=int(total),
                kcliques_per_s=total / max((end - start) / 1e3, 1e-9))
