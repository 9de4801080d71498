"""Host-side pieces of the serving loop: seeded Poisson arrivals and the
summary statistics (no GPU)."""
import numpy as np

from paper_2203_14906_amd import serve


def test_poisson_requests_seeded_and_rate():
    a = serve.poisson_requests(1000.0, 2.0, 36, seed=9)
    b = serve.poisson_requests(1000.0, 2.0, 36, seed=9)
    assert [(r.arrival, r.frame, r.order) for r in a] == [(r.arrival, r.frame, r.order) for r in b]
    assert 1800 < len(a) < 2200                      # ~ rate * duration
    t = np.array([r.arrival for r in a])
    assert np.all(np.diff(t) > 0) and t[-1] < 2.0
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1e-3) < 1e-4            # exponential gaps, mean 1/rate
    assert {r.order for r in a} == set(range(1, 7))
    assert all(0 <= r.frame < 36 for r in a)


def test_stats_summary():
    st = serve.ServeStats("batched", 4, 2.0, latencies_ms=np.array([1.0, 2.0, 3.0, 10.0]), launches=2)
    s = st.summary()
    assert s["frames_per_s"] == 2.0 and s["launches"] == 2
    assert s["p50_ms"] == 2.5 and abs(s["p99_ms"] - 9.79) < 1e-9
