"""Global rigid alignment: Gaussian pyramid + random rotation search + CSNGF over all shifts.

The search of Sec. 3.2: at level k both volumes are blurred with sigma_k and downsampled by
d_k; candidate rotations are the starting points of the level plus a_k random Euler
perturbations theta = theta_bar + U(-u_k, u_k)^3 (degrees; theta_bar drawn uniformly from
the starting points; rotation about x, then the resulting y, then the resulting z); every
candidate is scored at all displacements with the HIP path and the best p_{k+1} become the
next level's starting points.  The schedule of the paper's experiments (Sec. 3.2 and, for
the NGF methods' sigma, Sec. 5.1) is PAPER_SCHEDULE.

Host logic only: smoothing, downsampling and every evaluation run in libcsngf (C ABI).  The
evaluator is pluggable so that tests can drive the same search with the FP64 oracle.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import synth

PAPER_SCHEDULE = {
    "sigma": (5.0, 3.0, 2.0, 1.5),   # Gaussian sigma per level (voxels), NGF methods
    "d": (4, 2, 2, 1),               # downsampling factor per level
    "u": (180.0, 30.0, 10.0, 0.0),   # maximum random step per Euler angle (degrees)
    "a": (5000, 3000, 300, 0),       # random rotations per level
    "p": (1, 20, 3, 1),              # starting points per level
    "start": ((0.0, 0.0, 0.0),),     # initial starting point(s)
}


@dataclass
class LevelLog:
    d: int
    sigma: float
    shape: tuple
    candidates: int
    seconds: float
    best_score: float


@dataclass
class AlignResult:
    euler_deg: tuple          # best (theta_x, theta_y, theta_z)
    R: np.ndarray             # its inverse-mapping matrix
    shift: tuple              # displacement (chi_x, chi_y, chi_z) at full resolution
    score: float
    seconds: float
    levels: list = field(default_factory=list)

    def transform(self, A_shape_zyx, B_shape_zyx):
        return corner_transform(self.R, self.shift, B_shape_zyx)


def candidates(starts, u, a, rng):
    """The starting points themselves (re-scored, Sec. 3.2) followed by a random perturbations,
    each of a starting point drawn uniformly (drawn as arrays: a level has thousands)."""
    starts = [tuple(float(v) for v in s) for s in starts]
    a = int(a)
    if a <= 0:
        return list(starts)
    idx = rng.integers(0, len(starts), size=a)
    pert = np.asarray(starts, dtype=np.float64)[idx] + rng.uniform(-u, u, size=(a, 3))
    return starts + [tuple(row) for row in pert.tolist()]


def top_p(scores, p):
    """Indices of the p best scores; ties keep the lower index (stable order)."""
    scores = np.asarray(scores, dtype=np.float64)
    order = np.argsort(-scores, kind="stable")
    return [int(i) for i in order[:p]]


def corner_transform(R, shift, B_shape_zyx):
    """Map from A's voxel coordinates (x, y, z) to B's: x -> R (x + chi - c_B) + c_B."""
    nz, ny, nx = B_shape_zyx
    c = (np.array([nx, ny, nz], dtype=np.float64) - 1.0) / 2.0
    R = np.asarray(R, dtype=np.float64)
    chi = np.asarray(shift, dtype=np.float64)
    return lambda X: (np.asarray(X, dtype=np.float64) + chi - c) @ R.T + c


def corner_distance(A_shape_zyx, B_shape_zyx, R_true, shift_true, R_found, shift_found):
    """d_E of Sec. 5.1: mean Euclidean distance between the 8 corners of A's block mapped by
    the true and by the recovered transform (voxels)."""
    nz, ny, nx = A_shape_zyx
    X = np.array([[x, y, z] for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)], dtype=np.float64)
    t1 = corner_transform(R_true, shift_true, B_shape_zyx)(X)
    t2 = corner_transform(R_found, shift_found, B_shape_zyx)(X)
    return float(np.mean(np.linalg.norm(t1 - t2, axis=1)))


class GpuEvaluator:
    """Scores candidate rotations of one pyramid level with libcsngf (device-resident volumes).

    tune: run the library's autotuner once per pair of level shapes (FFT size, rotation slots,
    launch shapes; a few hundred milliseconds per shape, cached for later alignments) and
    evaluate with its choice; the scores do not depend on it."""

    def __init__(self, measure="squared", gamma=0.5, eps=1e-5, device="cuda:0", tune=False):
        import torch
        from . import binding
        self.torch, self.bd = torch, binding
        self.measure, self.gamma, self.eps = measure, gamma, eps
        self.device = torch.device(device)
        self.tune = tune
        self.tuned = {}   # (A level shape, B level shape) -> Context keywords

    def level(self, A, B, sigma, d):
        tA = A if not isinstance(A, np.ndarray) else self.torch.from_numpy(np.ascontiguousarray(A)).to(self.device)
        tB = B if not isinstance(B, np.ndarray) else self.torch.from_numpy(np.ascontiguousarray(B)).to(self.device)
        if sigma > 0 or d > 1:
            tA = self.bd.smooth_downsample(tA, sigma, d)
            tB = self.bd.smooth_downsample(tB, sigma, d)
        return tA, tB

    def score(self, Ak, Bk, Rs):
        # a level with few candidates (the last re-scores 1) needs no more rotation slots than
        # it has rotations; otherwise the library sizes the slots, or the tuned choice does
        kw = {"batch": len(Rs) if len(Rs) < 16 else 0}
        if self.tune and len(Rs) >= 16:
            key = (tuple(Ak.shape), tuple(Bk.shape))
            if key not in self.tuned:
                self.tuned[key] = self.bd.autotune(Ak, Bk, n_probe=64, measure=self.measure, gamma=self.gamma,
                                                   eps=self.eps, graphs=True)[0]
            kw = dict(self.tuned[key])
        # (graph replay: a level runs tens of identical launch sequences)
        with self.bd.Context(Ak, self.bd.dims_of(Bk), gamma=self.gamma, eps=self.eps, measure=self.measure,
                             graphs=True, **kw) as ctx:
            per, _ = ctx.evaluate(Bk, Rs)
        return ([p.score if p.valid else -np.inf for p in per], [tuple(p.shift) for p in per])


def align(A, B, schedule=PAPER_SCHEDULE, seed=0, evaluator=None):
    """Global rigid alignment of B onto A (Sec. 3.2).  Returns the best rotation, its
    full-resolution displacement and score, with per-level timings."""
    ev = evaluator if evaluator is not None else GpuEvaluator()
    rng = np.random.default_rng(seed)
    starts = [tuple(s) for s in schedule["start"]]
    t0 = time.perf_counter()
    levels = []
    m = len(schedule["d"])
    best = None
    for k in range(m):
        tl = time.perf_counter()
        d, sigma, u, a = schedule["d"][k], schedule["sigma"][k], schedule["u"][k], schedule["a"][k]
        Ak, Bk = ev.level(A, B, sigma, d)
        thetas = candidates(starts, u, a, rng)
        Rs = synth.euler_xyz_matrices(thetas)
        scores, shifts = ev.score(Ak, Bk, Rs)
        p_next = schedule["p"][k + 1] if k + 1 < m else 1
        keep = top_p(scores, p_next)
        starts = [thetas[i] for i in keep]
        b = keep[0]
        best = (thetas[b], Rs[b], shifts[b], scores[b], d)
        levels.append(LevelLog(d, sigma, tuple(Ak.shape), len(thetas), time.perf_counter() - tl, float(scores[b])))
    theta, R, shift, score, d = best
    full_shift = tuple(int(v) * d for v in shift)
    return AlignResult(tuple(theta), R, full_shift, float(score), time.perf_counter() - t0, levels)
