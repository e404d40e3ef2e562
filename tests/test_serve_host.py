"""Host side of the served form (no GPU): the seeded Poisson request stream and the latency summary."""
import numpy as np

from paper_2311_13798_amd.serve import poisson_requests, summarize


def test_poisson_stream_is_seeded_and_shaped():
    a = poisson_requests(rate=200.0, count=20000, n_graphs=7, k_lo=3, k_hi=12, seed=5)
    assert a == poisson_requests(rate=200.0, count=20000, n_graphs=7, k_lo=3, k_hi=12, seed=5)
    assert a != poisson_requests(rate=200.0, count=20000, n_graphs=7, k_lo=3, k_hi=12, seed=6)
    t = np.array([x[0] for x in a])
    assert t[0] == 0.0 and (np.diff(t) >= 0).all()
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 200.0) < 0.05 / 200.0  # exponential gaps of mean 1/rate
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.05   # coefficient of variation 1
    g = np.array([x[1] for x in a])
    k = np.array([x[2] for x in a])
    assert set(g.tolist()) == set(range(7)) and set(k.tolist()) == set(range(3, 13))
    w = poisson_requests(rate=50.0, count=5000, n_graphs=3, weights=[1, 0, 3], seed=2)
    gw = np.bincount([x[1] for x in w], minlength=3)
    assert gw[1] == 0 and abs(gw[2] / gw.sum() - 0.75) < 0.03


def test_summary_of_results():
    res = [{"arrival_ms": float(i), "done_ms": float(i) + (i % 10) + 1.0, "count": 2} for i in range(1000)]
    s = summarize(res)
    lat = np.array([(i % 10) + 1.0 for i in range(1000)])
    assert s["requests"] == 1000 and s["kcliques"] == 2000
    assert s["p50_ms"] == float(np.percentile(lat, 50)) and s["p99_ms"] == float(np.percentile(lat, 99))
    assert abs(s["makespan_s"] - (999 + 10 - 0) / 1e3) < 1e-12
    assert abs(s["kcliques_per_s"] - 2000 / s["makespan_s"]) < 1e-6
