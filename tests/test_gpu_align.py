"""Pyramid level kernel and the global search on the HIP path."""
import sys

import numpy as np
import pytest
from scipy.ndimage import gaussian_filter

from paper_2110_10156_amd import align, synth
from paper_2110_10156_amd import binding as bd

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("sigma,d,shape", [(0.0, 2, (9, 10, 11)), (1.5, 1, (20, 21, 22)), (5.0, 4, (40, 44, 30)),
                                           (2.0, 2, (33, 17, 8)), (3.0, 3, (7, 50, 13))])
def test_smooth_downsample_matches_scipy(sigma, d, shape):
    import torch
    rng = np.random.default_rng(int(sigma * 10) + d)
    vol = rng.random(shape).astype(np.float32)
    _say("blur", sigma, d, shape)
    out = bd.smooth_downsample(vol, sigma, d)
    ref = vol.astype(np.float64)
    if sigma > 0:
        ref = gaussian_filter(ref, sigma, mode="nearest", truncate=4.0)
    ref = ref[::d, ::d, ::d]
    assert out.shape == ref.shape
    assert np.max(np.abs(out - ref)) <= 1e-6 * max(1.0, float(np.max(np.abs(vol))))
    dev = bd.smooth_downsample(torch.from_numpy(vol).cuda(), sigma, d)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), out)


def test_gpu_search_matches_oracle_driven_search():
    from test_align_cpu import OracleEvaluator
    pair = synth.config0()
    rng = np.random.default_rng(8)
    B = pair.B
    sched = {"sigma": (1.0, 0.0), "d": (2, 1), "u": (25.0, 4.0), "a": (40, 12), "p": (1, 3, 1),
             "start": ((0.0, 0.0, 0.0),)}
    g = align.align(pair.A, B, sched, seed=3)
    o = align.align(pair.A, B, sched, seed=3, evaluator=OracleEvaluator())
    _say("search gpu", g.euler_deg, g.shift, g.score, "oracle", o.euler_deg, o.shift, o.score)
    assert g.euler_deg == o.euler_deg and g.shift == o.shift
    assert abs(g.score - o.score) <= 1e-4
    del rng


def test_paper_schedule_recovers_config1_transform():
    """The paper's schedule (Sec. 3.2) on the 96x96x64 pair (rotation <= 30 deg about a random
    axis, shift <= 15): success in the sense of Sec. 5.1, d_E < 5 voxels."""
    pair = synth.config1(n_random=0)
    res = align.align(pair.A, pair.B, align.PAPER_SCHEDULE, seed=0)
    dE = align.corner_distance(pair.A.shape, pair.B.shape, pair.true_rotation, pair.true_shift, res.R, res.shift)
    _say("config1 paper schedule", res.euler_deg, res.shift, "true", pair.true_shift, "dE", dE, "s", res.seconds,
         [(l.d, l.candidates, round(l.seconds, 3)) for l in res.levels])
    assert dE < 5.0
