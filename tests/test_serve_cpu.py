"""Host-side scheduling of the serving loop, on the CPU: admission by footprint, the
context cache (hits, least-recently-used eviction of idle contexts only), overlap of
requests in flight, latency accounting and the per-hit/miss summary.  The library
contexts are replaced by stand-ins that finish after a set time on a manual clock, so
only the server's own logic runs here (the device path is covered by the GPU tests).
"""
import numpy as np
import pytest

from paper_2110_10156_amd import serve

SPEC, PER_SLOT = 1000, 10          # bytes of a context's spectra, bytes per rotation slot


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeContext:
    made = []

    def __init__(self, A, dims_b, batch=0, graphs=False, measure="squared"):
        self.A, self.dims_b, self.batch = A, dims_b, batch
        self.finish_at = None
        self.closed = False
        self.evals = 0
        FakeContext.made.append(self)

    def evaluate_async(self, B, R):
        assert not self.closed and self.finish_at is None
        self.finish_at = CLOCK.t + DURATION
        self.evals += 1
        self.n = len(R)

    def done(self):
        return self.finish_at is not None and CLOCK.t >= self.finish_at

    def wait(self):
        assert self.done()
        self.finish_at = None
        return [None] * self.n, ("best", self.A)

    def close(self):
        self.closed = True


CLOCK = Clock()
DURATION = 1.0


@pytest.fixture(autouse=True)
def fake_library(monkeypatch):
    global CLOCK
    CLOCK = Clock()
    FakeContext.made = []
    monkeypatch.setattr(serve.bd, "Context", FakeContext)
    monkeypatch.setattr(serve.bd, "footprint", lambda da, db, measure="squared": (SPEC, PER_SLOT, (0, 0, 0)))
    yield


class Vol:
    def __init__(self, shape):
        self.shape = shape


def _server(budget, slot_budget=40):
    # slot_budget // PER_SLOT = 4 slots per context: a context needs SPEC + 40 bytes
    return serve.Server(budget, slot_budget=slot_budget, clock=CLOCK)


def _req(rid, key, shape=(8, 8, 8), n=5, arrival=0.0):
    return serve.Request(rid, key, Vol(shape), Vol(shape), np.zeros((n, 3, 3)), arrival)


def _advance(server, dt):
    CLOCK.t += dt
    server.poll()


NEED = SPEC + 4 * PER_SLOT


def test_cache_hit_reuses_the_idle_context():
    s = _server(10 * NEED)
    s.submit(_req(0, "a"))
    s.poll()
    assert len(FakeContext.made) == 1 and FakeContext.made[0].batch == 4
    _advance(s, DURATION)
    s.submit(_req(1, "a"))
    s.poll()
    _advance(s, DURATION)
    assert [r.cache_hit for r in s.results] == [False, True]
    assert s.stats.created == 1 and s.stats.hits == 1 and s.used == NEED
    # same fixed volume but another moving shape: another context
    s.submit(_req(2, "a", shape=(8, 8, 6)))
    s.poll()
    assert s.stats.created == 2 and s.used == 2 * NEED


def test_busy_context_is_not_shared_and_requests_overlap():
    s = _server(10 * NEED)
    s.submit(_req(0, "a"))
    s.submit(_req(1, "a"))
    s.poll()
    # the first context is busy, so the second request gets its own and both run at once
    assert s.stats.created == 2 and len(s.running) == 2 and s.stats.peak_inflight == 2
    _advance(s, DURATION)
    assert len(s.results) == 2 and all(not r.cache_hit for r in s.results)


def test_admission_waits_for_memory_then_evicts_least_recently_used():
    s = _server(2 * NEED)
    s.submit(_req(0, "a"))
    s.submit(_req(1, "b"))
    s.poll()
    assert s.used == 2 * NEED and len(s.running) == 2
    s.submit(_req(2, "c"))
    s.poll()
    # both contexts busy: nothing can be evicted, so "c" waits in the queue
    assert len(s.waiting) == 1 and s.stats.evicted == 0
    CLOCK.t += 0.5
    s.poll()
    assert len(s.waiting) == 1
    # "a" and "b" finish; "a" was used first, so it is the one evicted for "c"
    _advance(s, 0.5)
    assert len(s.waiting) == 0 and s.stats.evicted == 1
    ctx_a, ctx_b, ctx_c = FakeContext.made
    assert ctx_a.closed and not ctx_b.closed and not ctx_c.closed
    assert s.used == 2 * NEED and s.stats.peak_bytes == 2 * NEED
    _advance(s, DURATION)
    lat = {r.rid: r.latency for r in s.results}
    assert lat[0] == pytest.approx(1.0) and lat[1] == pytest.approx(1.0) and lat[2] == pytest.approx(2.0)
    starts = {r.rid: r.start for r in s.results}
    assert starts[2] == pytest.approx(1.0)


def test_arrival_order_is_kept_behind_a_waiting_request():
    s = _server(NEED)
    s.submit(_req(0, "a"))
    s.poll()
    s.submit(_req(1, "b"))   # needs "a" evicted, which is busy
    s.submit(_req(2, "a"))   # would hit "a" once idle, but arrives after "b"
    s.poll()
    assert [r.rid for r in s.waiting] == [1, 2]
    _advance(s, DURATION)    # "a" idle: "b" evicts it and runs; "2" then waits for memory
    assert [r.rid for r in s.waiting] == [2] and FakeContext.made[0].closed
    _advance(s, DURATION)
    _advance(s, DURATION)
    assert sorted(r.rid for r in s.results) == [0, 1, 2]
    assert s.stats.created == 3 and s.stats.evicted == 2


def test_request_above_the_budget_is_refused():
    s = _server(NEED - 1)
    s.submit(_req(0, "a"))
    with pytest.raises(RuntimeError, match="above the server budget"):
        s.poll()


def test_close_drains_and_releases_every_context():
    s = _server(10 * NEED)
    for i, k in enumerate("abc"):
        s.submit(_req(i, k))
    s.poll()
    CLOCK.t += DURATION   # every evaluation is due: close() must collect them before closing
    s.close()
    assert len(s.results) == 3 and all(c.closed for c in FakeContext.made) and s.used == 0


def test_summary_splits_hits_and_misses():
    R = serve.Result
    res = [R(0, [], None, 0.0, 0.0, 0.010, False), R(1, [], None, 0.5, 0.5, 0.520, True),
           R(2, [], None, 1.0, 1.0, 1.030, True), R(3, [], None, 1.5, 1.6, 1.640, False)]
    s = serve.summarize(res, rotations_per_request=200)
    assert s["requests"] == 4 and s["cache_hits"] == 2
    assert s["hits"]["n"] == 2 and s["misses"]["n"] == 2
    assert s["hits"]["p50_ms"] == pytest.approx(25.0) and s["misses"]["p50_ms"] == pytest.approx(75.0)
    assert s["p50_ms"] == pytest.approx(np.percentile([10, 20, 30, 140], 50))
    assert s["rotations_per_s"] == pytest.approx(4 * 200 / 1.64, rel=1e-3)


def test_poisson_arrivals_are_increasing_at_the_stated_rate():
    t = serve.poisson_arrivals(rate=20.0, n=20000, seed=3)
    assert np.all(np.diff(t) > 0)
    assert 20000 / t[-1] == pytest.approx(20.0, rel=0.03)
    np.testing.assert_array_equal(t, serve.poisson_arrivals(rate=20.0, n=20000, seed=3))
