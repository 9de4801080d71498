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


# --- the scheduler over a fake executor and a simulated clock (no GPU) -------

from types import SimpleNamespace  # noqa: E402


class FakeClock:
    """Simulated seconds: every reading advances time a little; sleeping
    advances it by the slept amount."""

    def __init__(self, step=2e-6):
        self.t, self.step = 0.0, step

    def __call__(self):
        self.t += self.step
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor:
    """Launch slots whose work completes `latency` simulated seconds after the
    launch; a launch that contains a request id in `refuse` is refused before
    anything is enqueued, as the library refuses a bad request."""

    def __init__(self, clock, n_slots=2, latency=1e-3, refuse=()):
        self.clock, self.latency, self.refuse = clock, latency, set(refuse)
        self.n_slots = n_slots
        self.launched = []           # (slot, [rid], time)
        self.busy = [0.0] * n_slots

    def launch(self, slot, reqs):
        if any(r.rid in self.refuse for r in reqs):
            raise serve.LaunchError("refused")
        assert self.busy[slot] <= self.clock.t, "slot reused while busy"
        self.launched.append((slot, [r.rid for r in reqs], self.clock.t))
        self.busy[slot] = self.clock.t + self.latency
        return self.busy[slot]

    def done(self, handle):
        return self.clock.t >= handle


def _pool(n=4):
    return SimpleNamespace(frames=[SimpleNamespace(side=32, n_elements=16, n_samples=256) for _ in range(n)])


def _server(pool, ex, clock, **kw):
    return serve.Server(None, pool, executor=ex, clock=clock, sleep=clock.sleep, **kw)


def _burst(n, t=1e-3, **kw):
    return [serve.Request(rid=i, arrival=t, frame=i % 4, order=1 + i % 6, **kw) for i in range(n)]


def test_budget_exhaustion_serialises_without_losing_requests():
    clock, pool = FakeClock(), _pool()
    one = 32 * 32 * 4 + 16 * 256 * 2
    ex = FakeExecutor(clock, n_slots=3, latency=5e-4)
    st = _server(pool, ex, clock, budget_bytes=one).run(_burst(12))
    assert st.admission_waits > 0 and st.max_inflight == 1      # the budget holds one frame
    assert sorted(rid for _, rids, _ in ex.launched for rid in rids) == list(range(12))
    assert st.summary()["rejected"] == st.summary()["dropped"] == st.summary()["failed"] == 0
    assert len(st.latencies_ms) == 12


def test_invalid_requests_are_rejected_alone():
    clock, pool = FakeClock(), _pool()
    ex = FakeExecutor(clock)
    reqs = _burst(8)
    reqs[1].order, reqs[3].order, reqs[5].frame, reqs[6].frame = 0, 7, -1, 99
    st = _server(pool, ex, clock).run(reqs)
    assert {r.rid for r in reqs if r.status == "rejected"} == {1, 3, 5, 6}
    assert {r.rid for r in reqs if r.status == "done"} == {0, 2, 4, 7}
    launched = {rid for _, rids, _ in ex.launched for rid in rids}
    assert launched == {0, 2, 4, 7} and st.rejected == 4 and len(st.latencies_ms) == 4


def test_deadlines_drop_only_late_requests():
    clock, pool = FakeClock(), _pool()
    ex = FakeExecutor(clock, n_slots=1, latency=5e-3)
    # one slot, max_batch 2: the first pair launches at once, the rest wait 5 ms
    # per pair against a 6 ms deadline -- the second pair makes it, the others drop
    reqs = _burst(8, deadline=6e-3)
    st = _server(pool, ex, clock, max_batch=2).run(reqs)
    done = [r.rid for r in reqs if r.status == "done"]
    dropped = [r.rid for r in reqs if r.status == "dropped"]
    assert done == [0, 1, 2, 3] and dropped == [4, 5, 6, 7] and st.dropped == 4
    assert not {rid for _, rids, _ in ex.launched for rid in rids} & set(dropped)
    assert all((r.done - r.arrival) * 1e3 <= 6.0 + 5.1 for r in reqs if r.status == "done")


def test_a_refused_request_fails_alone():
    clock, pool = FakeClock(), _pool()
    ex = FakeExecutor(clock, n_slots=2, refuse={3})
    reqs = _burst(6)
    st = _server(pool, ex, clock).run(reqs)
    assert [r.status for r in reqs] == ["done", "done", "done", "failed", "done", "done"]
    assert st.failed == 1 and reqs[3].image is None
    # the refused batch was relaunched one request at a time
    assert all(len(rids) == 1 for _, rids, _ in ex.launched)
    assert sorted(rid for _, rids, _ in ex.launched for rid in rids) == [0, 1, 2, 4, 5]


def test_requests_per_launch_are_reported():
    clock, pool = FakeClock(), _pool()
    ex = FakeExecutor(clock, n_slots=1, latency=5e-3)
    # one slot, max_batch 3: a burst of 8 goes out as 3 + 3 + 2
    st = _server(pool, ex, clock, max_batch=3).run(_burst(8))
    assert st.batch_sizes == [len(rids) for _, rids, _ in ex.launched] == [3, 3, 2]
    s = st.summary()["requests_per_launch"]
    assert s["max"] == 3 and abs(s["mean"] - 8 / 3) < 0.01
    assert s["histogram"] == {"2-3": 3}
    assert serve.ServeStats("x", 0, 0.0, batch_sizes=[1, 1, 4, 9, 17, 40]).launch_histogram() == \
        {"1": 2, "4-7": 1, "8-15": 1, "16-31": 1, "32-63": 1}
