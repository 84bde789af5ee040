"""The largest supported volumes: 256^3 on both sides, FFT 512^3 (every axis at the longest
compile-time plan, 512 = 2^9; 16.8 Mvoxel, five times the paper-scale pair).  The oracle's
whole FP64 map at this size is out of reach in a test, so the GPU's per-rotation results are
checked against Eq. (5) summed directly by the oracle at the reported displacement (N exact,
|dC| <= 1e-4, gamma rule) and at its six neighbours, and B, a translated noisy copy of A,
must give back the translation at the identity rotation.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2110_10156_amd import binding as bd
from paper_2110_10156_amd import synth

pytestmark = pytest.mark.gpu

CTOL = 1e-4
N = 256
SHIFT = (7, -5, 11)   # (x, y, z): B(y) = A(y - t) on the overlap


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _pair():
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(256)
    big = gaussian_filter(rng.random((N + 32,) * 3).astype(np.float32), 2.5)
    big = (big - big.min()) / (big.max() - big.min())
    tx, ty, tz = SHIFT
    A = np.ascontiguousarray(big[16:16 + N, 16:16 + N, 16:16 + N])
    B = np.ascontiguousarray(big[16 - tz:16 - tz + N, 16 - ty:16 - ty + N, 16 - tx:16 - tx + N])
    B = (B + rng.normal(0.0, 0.005, B.shape)).astype(np.float32)
    return A, B


def test_maximum_extent_256_cubed():
    A, B = _pair()
    rots = np.stack([np.eye(3), synth.axis_angle_matrix(np.array([0.3, -0.5, 0.8]), math.radians(6.0))])
    with bd.Context(A, bd.dims_of(B)) as ctx:
        info = ctx.info()
        _say("256^3: P", tuple(info.pad), "slots", info.batch, "spectra MiB", info.spectra_bytes >> 20)
        assert tuple(info.pad) == (512, 512, 512)
        per, best = ctx.evaluate(B, rots)
    assert best.rot_index == 0 and tuple(best.shift) == SHIFT, (best.rot_index, tuple(best.shift))
    fa = O.fixed_fields(A)
    count_a = int(fa.mask.sum())
    for i, g in enumerate(per):
        assert g.valid, i
        fb = O.moving_fields(B, O.quantize_rotation(rots[i]))
        thr = 0.5 * min(count_a, int(fb.mask.sum()))
        S, n = O.similarity_at(fa, fb, tuple(g.shift))
        assert g.overlap == n and n >= thr, (i, g.overlap, n, thr)
        assert abs(float(g.score) - S / n) <= CTOL, (i, float(g.score), S / n)
        # the reported displacement beats its valid neighbours (Eq. (5) summed directly)
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            chi = tuple(a + b for a, b in zip(g.shift, d))
            S2, n2 = O.similarity_at(fa, fb, chi)
            if n2 >= max(1, thr):
                assert S2 / n2 <= float(g.score) + CTOL, (i, chi, S2 / n2, float(g.score))
        _say("rotation", i, "shift", tuple(g.shift), "score", float(g.score), "N", n)
