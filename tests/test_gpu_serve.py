"""Serving loop: results are the same alone and in the mix; the cache and admission work."""
import sys

import numpy as np
import pytest

from paper_2110_10156_amd import binding as bd
from paper_2110_10156_amd import serve, synth
from parity_util import check_against_oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _pool(torch):
    dev = torch.device("cuda:0")
    pairs = {"c16": synth.cube_pair(16), "c24": synth.cube_pair(24), "c0": synth.config0(),
             "m48": synth.mixed_pair_of_size((48, 48, 48))}
    return {k: (torch.from_numpy(p.A).to(dev), torch.from_numpy(p.B).to(dev)) for k, p in pairs.items()}


def test_served_mix_equals_each_request_alone():
    import torch
    vols = _pool(torch)
    keys = ["c16", "c24", "c0", "m48", "c16", "c0", "m48", "c24"]
    reqs = [serve.Request(i, k, vols[k][0], vols[k][1], synth.random_rotations(12 + 3 * i, 900 + i))
            for i, k in enumerate(keys)]
    srv = serve.Server(hbm_budget=6 << 30, slot_budget=1 << 28)
    res = serve.run_stream(srv, lambda i: reqs[i], np.zeros(len(reqs)))   # all arrive at once
    assert [r.rid for r in res] == list(range(len(reqs)))
    assert srv.stats.peak_inflight >= 2
    _say("mix", srv.stats.created, "contexts,", srv.stats.hits, "hits, peak in flight", srv.stats.peak_inflight)
    srv.close()
    for req, r in zip(reqs, res):
        with bd.Context(req.A, bd.dims_of(req.B)) as c:        # alone, plain path, other slot count
            per, best = c.evaluate(req.B, req.rotations)
        assert best.rot_index == r.best.rot_index
        for a, b in zip(per, r.per):
            assert a.score == b.score and tuple(a.shift) == tuple(b.shift) and a.overlap == b.overlap
        # and each served result against the oracle
        _say("served request", req.rid, "vs oracle", tuple(req.A.shape))
        check_against_oracle(req.A.cpu().numpy(), req.B.cpu().numpy(), req.rotations, r.per, r.best,
                             P=bd.footprint(bd.dims_of(req.A), bd.dims_of(req.B))[2])


def test_admission_by_footprint_and_eviction():
    import torch
    vols = _pool(torch)
    spec, slot, _ = bd.footprint((48, 48, 48), (48, 48, 48))
    budget = spec + 2 * slot + 1                      # room for exactly one 48^3 context with 2 slots
    srv = serve.Server(hbm_budget=budget, slot_budget=2 * slot)
    keys = ["m48", "c16", "m48"]
    reqs = [serve.Request(i, k, vols[k][0], vols[k][1], synth.random_rotations(10, 50 + i)) for i, k in enumerate(keys)]
    res = serve.run_stream(srv, lambda i: reqs[i], np.zeros(3))
    assert len(res) == 3 and srv.used <= budget
    assert srv.stats.evicted >= 1                     # the 16^3 pair needed the 48^3 context's room
    srv.close()


def test_poisson_stream_reports_latency():
    import torch
    vols = _pool(torch)
    keys = list(vols)
    rng = np.random.default_rng(3)
    srv = serve.Server(hbm_budget=8 << 30, slot_budget=1 << 28)
    arr = serve.poisson_arrivals(50.0, 30, seed=4)
    res = serve.run_stream(srv, lambda i: serve.Request(i, keys[i % len(keys)], *vols[keys[i % len(keys)]],
                                                        synth.random_rotations(32, 400 + i)), arr)
    s = serve.summarize(res, 32)
    _say("poisson 50/s", s)
    assert s["requests"] == 30 and s["p99_ms"] >= s["p50_ms"] > 0 and s["cache_hits"] > 0
    srv.close()
    del rng
