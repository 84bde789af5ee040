"""Continuous-batching alignment server on libcsngf.

Requests (fixed volume A, moving volume B, candidate rotations) arrive over time.  The
server keeps contexts - A's resident spectra plus rotation workspaces - in a device cache
keyed by the fixed volume and B's shape, admits a request as soon as a context for it is
idle or a new one fits the HBM budget (idle contexts are evicted least-recently-used), and
puts every admitted request's evaluation in flight on its context's own stream.  Requests
that arrive while others run therefore overlap with them on the device.  Per request the
server records arrival, start and finish times; latency is finish - arrival.

Host-side scheduling only: every evaluation runs in the HIP library (asynchronous C ABI).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as bd


@dataclass
class Request:
    rid: int
    key: str                 # identity of the fixed volume (spectra cache key)
    A: object                # fixed volume (device tensor)
    B: object                # moving volume (device tensor)
    rotations: np.ndarray    # (n, 3, 3)
    arrival: float = 0.0     # seconds on the server clock


@dataclass
class Result:
    rid: int
    per: list
    best: object
    arrival: float
    start: float
    finish: float
    cache_hit: bool

    @property
    def latency(self):
        return self.finish - self.arrival


@dataclass
class _Slot:
    key: tuple
    ctx: object
    nbytes: int
    busy: bool = False
    last_used: float = 0.0


@dataclass
class Stats:
    created: int = 0
    evicted: int = 0
    hits: int = 0
    peak_bytes: int = 0
    peak_inflight: int = 0
    inflight_samples: list = field(default_factory=list)


class Server:
    """hbm_budget: bytes of device memory the cached contexts may hold in total;
    slot_budget: workspace bytes per context (sets its rotation slots)."""

    def __init__(self, hbm_budget, slot_budget=4 << 30, graphs=True, measure="squared", clock=time.perf_counter):
        self.budget = int(hbm_budget)
        self.slot_budget = int(slot_budget)
        self.graphs = graphs
        self.measure = measure
        self.clock = clock
        self.t0 = clock()
        self.pool = collections.OrderedDict()   # key -> list of _Slot
        self.used = 0
        self.waiting = collections.deque()
        self.running = []                       # (Request, _Slot, start, hit)
        self.results = []
        self.stats = Stats()

    def now(self):
        return self.clock() - self.t0

    def submit(self, req: Request):
        self.waiting.append(req)

    # ------------------------------------------------------------------ cache
    def _evict_one(self):
        for key, slots in self.pool.items():
            for s in slots:
                if not s.busy:
                    slots.remove(s)
                    s.ctx.close()
                    self.used -= s.nbytes
                    self.stats.evicted += 1
                    if not slots:
                        del self.pool[key]
                    return True
        return False

    def _acquire(self, req):
        key = (req.key, tuple(req.B.shape))
        for s in self.pool.get(key, []):
            if not s.busy:
                self.pool.move_to_end(key)
                self.stats.hits += 1
                return s, True
        dims_b = bd.dims_of(req.B)
        spec, per_slot, _ = bd.footprint(bd.dims_of(req.A), dims_b, measure=self.measure)
        batch = int(max(1, min(64, self.slot_budget // per_slot)))
        need = spec + batch * per_slot
        if need > self.budget:
            raise RuntimeError(f"request {req.rid} needs {need} bytes, above the server budget")
        while self.used + need > self.budget:
            if not self._evict_one():
                return None, False
        ctx = bd.Context(req.A, dims_b, batch=batch, graphs=self.graphs, measure=self.measure)
        s = _Slot(key, ctx, need)
        self.pool.setdefault(key, []).append(s)
        self.pool.move_to_end(key)
        self.used += need
        self.stats.created += 1
        self.stats.peak_bytes = max(self.stats.peak_bytes, self.used)
        return s, False

    # ------------------------------------------------------------------ loop
    def poll(self):
        """Collect finished evaluations, then admit waiting requests in arrival order."""
        progressed = False
        still = []
        for req, slot, start, hit in self.running:
            if slot.ctx.done():
                per, best = slot.ctx.wait()
                t = self.now()
                slot.busy = False
                slot.last_used = t
                self.results.append(Result(req.rid, per, best, req.arrival, start, t, hit))
                progressed = True
            else:
                still.append((req, slot, start, hit))
        self.running = still
        while self.waiting:
            req = self.waiting[0]
            slot, hit = self._acquire(req)
            if slot is None:
                break
            self.waiting.popleft()
            slot.busy = True
            slot.ctx.evaluate_async(req.B, req.rotations)
            self.running.append((req, slot, self.now(), hit))
            progressed = True
        self.stats.peak_inflight = max(self.stats.peak_inflight, len(self.running))
        return progressed

    def drain(self, idle_sleep=2e-4):
        while self.waiting or self.running:
            if not self.poll():
                time.sleep(idle_sleep)

    def close(self):
        self.drain()
        for slots in self.pool.values():
            for s in slots:
                s.ctx.close()
        self.pool.clear()
        self.used = 0


def poisson_arrivals(rate, n, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def run_stream(server: Server, make_request, arrivals, idle_sleep=2e-4):
    """Submit make_request(i) at arrivals[i] (seconds on the server clock, relative to the
    call) and serve until every request has finished; returns the results in rid order."""
    n = len(arrivals)
    base = server.now()
    i = 0
    first = len(server.results)
    while len(server.results) - first < n:
        t = server.now() - base
        while i < n and arrivals[i] <= t:
            req = make_request(i)
            req.arrival = base + float(arrivals[i])
            server.submit(req)
            i += 1
        server.stats.inflight_samples.append(len(server.running))
        if not server.poll():
            time.sleep(idle_sleep)
    return sorted(server.results[first:], key=lambda r: r.rid)


def summarize(results, rotations_per_request):
    """Latency percentiles (ms) over all requests and separately over cache hits and misses
    (a miss created a context: A's spectra were computed for it), and the sustained rate."""
    lat = np.array([r.latency for r in results]) * 1e3
    hit = np.array([r.cache_hit for r in results], dtype=bool)
    span = max(r.finish for r in results) - min(r.arrival for r in results)

    def pct(x):
        if x.size == 0:
            return None
        return {"n": int(x.size), "p50_ms": round(float(np.percentile(x, 50)), 2),
                "p99_ms": round(float(np.percentile(x, 99)), 2)}

    return {
        "requests": len(results),
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "mean_ms": round(float(lat.mean()), 2),
        "rotations_per_s": round(len(results) * rotations_per_request / span, 1),
        "cache_hits": int(hit.sum()),
        "hits": pct(lat[hit]),
        "misses": pct(lat[~hit]),
    }
