"""Seeded synthetic volume pairs and candidate rotations.

Input generation only: this module holds none of the similarity arithmetic (no gradients,
no normalized gradient fields, no correlation, no overlap counts).  Both the HIP path and
the FP64 oracle receive the arrays it produces.

The paper evaluates on brain volumes of four modalities (Sec. 4), cropped to 151^3 blocks,
displaced by a uniformly random rotation and an integer shift of up to 30 voxels per axis.
Those volumes are not available here; the generators below stand in for them with analytic
phantoms of the same size class (about 3.4 Mvoxel), the same shift range and a multimodal
intensity relation (a non-monotonic or permuted intensity map between the two volumes).

Conventions
-----------
* Volumes are float32 arrays in C order ``[nz][ny][nx]`` (x fastest).
* Coordinates are written ``(x, y, z)``; a 3x3 matrix ``R`` acts on such column vectors.
* A candidate rotation ``R`` maps an output voxel ``x`` on B's grid to the source point
  ``R (x - c) + c`` in B, ``c = (n - 1) / 2`` (inverse mapping, B resampled as B o T).
* A "true" transform ``(R*, chi*)`` is built so that resampling B with ``R*`` gives a
  volume whose structure sits at ``x - chi*``; the similarity is then maximal at the
  displacement ``chi*`` (A(x) is compared with the resampled B at ``x + chi``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "quat_to_matrix", "axis_angle_matrix", "euler_xyz_matrix", "euler_xyz_matrices", "random_rotations",
    "intensity_map_f", "VolumePair", "config0", "config1", "config2", "cube_pair",
    "mixed_pair", "mixed_pair_of_size", "MIXED_SHAPES",
]


# ----------------------------------------------------------------------------- rotations
def quat_to_matrix(q) -> np.ndarray:
    """Unit quaternion (w, x, y, z), Hamilton convention, to a 3x3 rotation matrix."""
    w, x, y, z = (float(v) for v in q)
    s = w * w + x * x + y * y + z * z
    w, x, y, z = (v / math.sqrt(s) for v in (w, x, y, z))
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ], dtype=np.float64)


def axis_angle_matrix(axis, angle_rad: float) -> np.ndarray:
    """Right-handed rotation by ``angle_rad`` about ``axis`` (Rodrigues)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    h = 0.5 * angle_rad
    return quat_to_matrix([math.cos(h), *(math.sin(h) * a)])


def euler_xyz_matrix(ax_deg: float, ay_deg: float, az_deg: float) -> np.ndarray:
    """Intrinsic Euler rotation: about x, then the resulting y, then the resulting z (Sec. 3.2).

    Intrinsic x-y'-z'' composes as ``Rx @ Ry @ Rz``.  Angles are in degrees (the step sizes
    of the pyramid schedule, up to 180, only make sense in degrees).
    """
    rx = axis_angle_matrix([1, 0, 0], math.radians(ax_deg))
    ry = axis_angle_matrix([0, 1, 0], math.radians(ay_deg))
    rz = axis_angle_matrix([0, 0, 1], math.radians(az_deg))
    return rx @ ry @ rz


def euler_xyz_matrices(angles_deg) -> np.ndarray:
    """euler_xyz_matrix for every row (theta_x, theta_y, theta_z) of an (n, 3) array of degrees,
    as one (n, 3, 3) array (the rotations about the three axes built in closed form)."""
    t = np.radians(np.asarray(angles_deg, dtype=np.float64).reshape(-1, 3))
    c, s = np.cos(t), np.sin(t)
    n = t.shape[0]
    one, zero = np.ones(n), np.zeros(n)
    rx = np.stack([np.stack([one, zero, zero], -1), np.stack([zero, c[:, 0], -s[:, 0]], -1),
                   np.stack([zero, s[:, 0], c[:, 0]], -1)], -2)
    ry = np.stack([np.stack([c[:, 1], zero, s[:, 1]], -1), np.stack([zero, one, zero], -1),
                   np.stack([-s[:, 1], zero, c[:, 1]], -1)], -2)
    rz = np.stack([np.stack([c[:, 2], -s[:, 2], zero], -1), np.stack([s[:, 2], c[:, 2], zero], -1),
                   np.stack([zero, zero, one], -1)], -2)
    return rx @ ry @ rz


def random_rotations(n: int, seed: int) -> np.ndarray:
    """``n`` uniformly random rotations: normalised 4-D Gaussian quaternions, shape (n, 3, 3)."""
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4))
    return np.stack([quat_to_matrix(v) for v in q]) if n else np.zeros((0, 3, 3))


def _random_axis(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


# ----------------------------------------------------------------------------- intensities
_F_KNOTS_X = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
_F_KNOTS_Y = np.array([0.1, 0.8, 0.3, 1.0, 0.0])


def intensity_map_f(v: np.ndarray) -> np.ndarray:
    """Fixed non-monotonic piecewise-linear intensity map on [0, 1] (second modality)."""
    return np.interp(v, _F_KNOTS_X, _F_KNOTS_Y)


# ----------------------------------------------------------------------------- phantoms
def _grid_points(shape_zyx):
    nz, ny, nx = shape_zyx
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return np.stack([x, y, z], axis=-1)  # (..., 3) in (x, y, z)


@dataclass
class _Blobs:
    mu: np.ndarray      # (k, 3) centres, (x, y, z)
    sigma: np.ndarray   # (k,)
    amp: np.ndarray     # (k,)

    def __call__(self, pts: np.ndarray) -> np.ndarray:
        px = np.ascontiguousarray(pts[..., 0])
        py = np.ascontiguousarray(pts[..., 1])
        pz = np.ascontiguousarray(pts[..., 2])
        out = np.zeros(px.shape, dtype=np.float64)
        d2 = np.empty_like(out)
        tmp = np.empty_like(out)
        for m, s, a in zip(self.mu, self.sigma, self.amp):
            np.subtract(px, m[0], out=d2)
            np.square(d2, out=d2)
            np.subtract(py, m[1], out=tmp)
            np.square(tmp, out=tmp)
            d2 += tmp
            np.subtract(pz, m[2], out=tmp)
            np.square(tmp, out=tmp)
            d2 += tmp
            d2 *= -1.0 / (2.0 * s * s)
            np.exp(d2, out=d2)
            d2 *= a
            out += d2
        return out


def _make_blobs(rng, n_blobs: int, extent_xyz) -> _Blobs:
    ext = np.asarray(extent_xyz, dtype=np.float64)
    mu = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * ext
    sigma = rng.uniform(2.0, 5.0, size=n_blobs)
    amp = rng.uniform(0.5, 1.0, size=n_blobs)
    return _Blobs(mu, sigma, amp)


@dataclass
class _ShellPhantom:
    """Four tissue classes: 0 background, 1 shell, 2 interior, 3 ellipsoidal blobs."""
    centre: np.ndarray
    outer: np.ndarray          # semi-axes of the outer ellipsoid (x, y, z)
    inner: np.ndarray          # semi-axes of the inner ellipsoid
    blob_c: np.ndarray         # (k, 3)
    blob_ax: np.ndarray        # (k, 3) semi-axes
    blob_rot: np.ndarray       # (k, 3, 3) orientation

    def labels(self, pts: np.ndarray) -> np.ndarray:
        lab = np.zeros(pts.shape[:-1], dtype=np.int8)
        d = pts - self.centre
        r_out = np.sum((d / self.outer) ** 2, axis=-1)
        r_in = np.sum((d / self.inner) ** 2, axis=-1)
        lab[r_out <= 1.0] = 1
        lab[r_in <= 1.0] = 2
        for c, ax, rot in zip(self.blob_c, self.blob_ax, self.blob_rot):
            local = (pts - c) @ rot      # coordinates in the blob frame
            inside = np.sum((local / ax) ** 2, axis=-1) <= 1.0
            lab[inside & (r_in <= 1.0)] = 3
        return lab


def _make_shell(rng, n_xyz) -> _ShellPhantom:
    n = np.asarray(n_xyz, dtype=np.float64)
    centre = (n - 1.0) / 2.0 + rng.uniform(-2.0, 2.0, size=3)
    outer = n * np.array([0.40, 0.44, 0.40]) * rng.uniform(0.95, 1.05, size=3)
    inner = outer - rng.uniform(4.0, 7.0, size=3)
    k = 14
    blob_c = centre + rng.uniform(-0.6, 0.6, size=(k, 3)) * inner
    blob_ax = rng.uniform(0.05, 0.15, size=(k, 3)) * n
    blob_rot = np.stack([quat_to_matrix(rng.normal(size=4)) for _ in range(k)])
    return _ShellPhantom(centre, outer, inner, blob_c, blob_ax, blob_rot)


# ----------------------------------------------------------------------------- pairs
@dataclass
class VolumePair:
    """A fixed volume A, a moving volume B, candidate rotations and the known truth."""
    name: str
    A: np.ndarray                       # float32 [nz][ny][nx]
    B: np.ndarray                       # float32 [nz][ny][nx]
    rotations: np.ndarray               # (n, 3, 3) float64, inverse-mapping matrices
    true_rotation: np.ndarray           # (3, 3)
    true_shift: tuple                   # (chi_x, chi_y, chi_z)
    true_index: int | None              # index of the true rotation in ``rotations``
    pad: tuple = (0, 0, 0)              # requested FFT size (Px, Py, Pz); 0 = automatic
    meta: dict = field(default_factory=dict)

    @property
    def dims_a(self):
        nz, ny, nx = self.A.shape
        return (nx, ny, nz)

    @property
    def dims_b(self):
        nz, ny, nx = self.B.shape
        return (nx, ny, nz)


def _source_points(shape_zyx, R_true, shift_xyz):
    """Points ``R*^-1 (y - c) + c - chi*`` for every voxel y of a grid of shape_zyx."""
    pts = _grid_points(shape_zyx)
    nz, ny, nx = shape_zyx
    c = (np.array([nx, ny, nz], dtype=np.float64) - 1.0) / 2.0
    Rinv = np.linalg.inv(R_true)
    return (pts - c) @ Rinv.T + c - np.asarray(shift_xyz, dtype=np.float64)


def config0(seed: int = 0) -> VolumePair:
    """32^3 pair: 20 Gaussian blobs; B = f(A shifted by t) + noise; identity rotation only."""
    rng = np.random.default_rng(seed)
    shape = (32, 32, 32)
    blobs = _make_blobs(rng, 20, (32, 32, 32))
    grid = _grid_points(shape)
    a_an = blobs(grid)
    amax = a_an.max()
    t = tuple(int(v) for v in rng.integers(-6, 7, size=3))
    b_src = blobs(grid - np.asarray(t, dtype=np.float64)) / amax
    noise = rng.normal(0.0, 0.01, size=shape)
    A = (a_an / amax).astype(np.float32)
    B = (intensity_map_f(b_src) + noise).astype(np.float32)
    R = np.eye(3)[None]
    return VolumePair("config0", A, B, R, np.eye(3), t, 0, pad=(64, 64, 64))


def config1(seed: int = 1, n_random: int = 128) -> VolumePair:
    """96x96x64 pair with 360 blobs, f-mapped B, rotation <= 30 deg about a random axis, shift <= 15."""
    rng = np.random.default_rng(seed)
    shape = (64, 96, 96)
    blobs = _make_blobs(rng, 360, (96, 96, 64))
    a_an = blobs(_grid_points(shape))
    amax = a_an.max()
    R_true = axis_angle_matrix(_random_axis(rng), math.radians(rng.uniform(0.0, 30.0)))
    t = tuple(int(v) for v in rng.integers(-15, 16, size=3))
    b_src = blobs(_source_points(shape, R_true, t)) / amax
    noise = rng.normal(0.0, 0.01, size=shape)
    A = (a_an / amax).astype(np.float32)
    B = (intensity_map_f(b_src) + noise).astype(np.float32)
    rots = np.concatenate([random_rotations(n_random, 101), R_true[None]], axis=0)
    return VolumePair("config1", A, B, rots, R_true, t, n_random, pad=(192, 192, 128))


def _shell_pair(name, rng, n_xyz, n_random, rot_seed, pad, max_angle_deg=60.0, max_shift=30,
                min_box_overlap=0.6):
    nx, ny, nz = n_xyz
    shape = (nz, ny, nx)
    ph = _make_shell(rng, n_xyz)
    lab_a = ph.labels(_grid_points(shape))
    int_a = np.array([0.0, 0.9, 0.4, 0.7])
    int_b = np.array([0.6, 0.0, 1.0, 0.3])
    # True transform: re-draw until the plain box-overlap fraction of the shift is large
    # enough that the truth comfortably meets the minimum-overlap rule.
    n = np.array(n_xyz, dtype=np.float64)
    while True:
        R_true = axis_angle_matrix(_random_axis(rng),
                                   math.radians(rng.uniform(0.0, max_angle_deg)))
        lim = np.minimum(max_shift, ((n - 2) // 3).astype(int))
        t = np.array([int(rng.integers(-l, l + 1)) for l in lim])
        frac = float(np.prod((n - 2 - np.abs(t)) / (n - 2)))
        if frac >= min_box_overlap:
            break
    lab_b = ph.labels(_source_points(shape, R_true, t))
    from scipy.ndimage import gaussian_filter
    b = gaussian_filter(int_b[lab_b], sigma=1.5, truncate=4.0, mode="nearest")
    b = b + rng.normal(0.0, 0.01, size=shape)
    A = int_a[lab_a].astype(np.float32)
    B = b.astype(np.float32)
    rots = np.concatenate([random_rotations(n_random, rot_seed), R_true[None]], axis=0)
    return VolumePair(name, A, B, rots, R_true, tuple(int(v) for v in t), n_random, pad=pad)


def config2(seed: int = 2, n_random: int = 1000) -> VolumePair:
    """176x176x110 (3.4 Mvoxel) 4-class shell phantom; B = permuted classes, smoothed, noisy.

    Rotation up to 60 deg, shift up to 30 voxels; ``n_random`` random rotations followed by
    the true one (index ``n_random``).
    """
    rng = np.random.default_rng(seed)
    return _shell_pair("config2", rng, (176, 176, 110), n_random, 102, (352, 352, 220))


MIXED_SHAPES = [(48, 48, 48), (64, 64, 48), (96, 96, 96), (128, 128, 96), (176, 176, 110)]


def mixed_pair(i: int, n_random: int = 256) -> VolumePair:
    """Pair ``i`` of the uneven-size batch: size uniform over MIXED_SHAPES, built as config2."""
    rng = np.random.default_rng(3000 + i)
    n_xyz = MIXED_SHAPES[int(rng.integers(0, len(MIXED_SHAPES)))]
    pad = tuple(2 * v for v in n_xyz)
    return _shell_pair(f"mixed{i}", rng, n_xyz, n_random, 3100 + i, pad)


def mixed_pair_of_size(n_xyz, seed: int = 3999, n_random: int = 0) -> VolumePair:
    """A pair of the given size built as config2 (4-class shell phantom, permuted, smoothed, noisy)."""
    rng = np.random.default_rng(seed)
    return _shell_pair(f"mixed{n_xyz[0]}x{n_xyz[1]}x{n_xyz[2]}", rng, tuple(n_xyz), n_random, seed + 1,
                       tuple(2 * v for v in n_xyz))


def cube_pair(side: int, seed: int = 7, n_random: int = 4) -> VolumePair:
    """Cube volumes of the given side (the per-evaluation timing sweep of Sec. 5.2)."""
    rng = np.random.default_rng(seed + side)
    shape = (side, side, side)
    nb = max(4, int(round(20 * side ** 3 / 32768)))
    blobs = _make_blobs(rng, nb, (side, side, side))
    a_an = blobs(_grid_points(shape))
    amax = a_an.max()
    t = tuple(int(v) for v in rng.integers(-(side // 5), side // 5 + 1, size=3))
    b_src = blobs(_grid_points(shape) - np.asarray(t, dtype=np.float64)) / amax
    A = (a_an / amax).astype(np.float32)
    B = (intensity_map_f(b_src) + rng.normal(0.0, 0.01, size=shape)).astype(np.float32)
    rots = np.concatenate([np.eye(3)[None], random_rotations(n_random - 1, seed)], axis=0)
    return VolumePair(f"cube{side}", A, B, rots, np.eye(3), t, 0, pad=(2 * side,) * 3)
