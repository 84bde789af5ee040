"""FP64 CPU oracle for the cross similarity of normalized gradient fields (CSNGF).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import this module.  The product path (the HIP library and its binding) never calls
it, and this module imports nothing from the product package.

What it computes, in the paper's order (Ofverstedt, Lindblad, Sladoje, "Cross-Sim-NGF"):

* Sec. 2, Eq. (1): regularised normalized gradient field  n = grad I / sqrt(|grad I|^2 + eps^2),
  eps = 1e-5.
* Sec. 2, Eq. (2): pointwise similarity  s = <n_A, n_B>^2.
* Sec. 3.1, Eq. (5): for every integer displacement chi,
  C(chi) = (1 / N(chi)) * sum_x M_A(x) M_B(x + chi) s(x; A(x), B(x + chi)),
  with N(chi) the number of overlapping mask voxels (the mask cross-correlation).
* Sec. 3.1, Eq. (6)-(8): the same sums through 6 separable products and frequency-domain
  cross-correlation (summed before one inverse transform).
* Sec. 2, Eq. (3) and Sec. 5.1 (USNGF): the unsquared variant s = <n_A, n_B>, whose three
  separable parts are the per-axis products (measure="unsquared").
* Sec. 3.2: B resampled under a candidate rotation by trilinear interpolation (inverse
  mapping), its NGF taken after resampling; only displacements meeting a minimum overlap
  gamma (0.5) count; zero padding makes the correlation linear; the best displacement per
  rotation is the argmax of C.

Readings where the paper is silent (each also listed in the design notes):

* Gradient: central differences, unit spacing, factor 1/2, no extrapolation; the mask is
  eroded by the 7-point stencil so every counted voxel has all six neighbours.
* Resampled-B mask: the source point lies in the closed box [0, n-1] per axis; with a user
  mask on B, all 8 corners of the source cell must lie in it.
* Rotation centre: B's geometric centre (n_B - 1) / 2; the resampled B lives on B's grid.
* Rotation matrices are quantised to multiples of 2^-16 (round half to even) before use,
  so that every source coordinate is exact in FP64 (and in fixed point on the GPU).
* Upper edge: the cell index is clamped to n - 2, so p = n - 1 gives weight 1 on the
  last sample.
* gamma reference: chi is valid iff N(chi) >= 1 and N(chi) >= gamma * min(|M_A|, |M_B^|).
* Displacement range: chi in [-(n_A - 1), n_B - 1] per axis; A(x) pairs with B^(x + chi).
* Ties: the larger C wins; equal C goes to the smaller canonical index (chi_z, chi_y, chi_x
  lexicographic, each ascending); across rotations the smaller rotation index wins.

Array conventions: volumes are ``[nz][ny][nx]`` (x fastest); coordinates and matrices use
(x, y, z) order; maps are ``[Wz][Wy][Wx]`` with W = n_A + n_B - 1 and index i = chi + n_A - 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

import os

# FFT worker threads: the CPU cores this process may use, at most 16.
try:
    WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
except AttributeError:  # pragma: no cover
    WORKERS = max(1, min(16, os.cpu_count() or 1))

EPS_DEFAULT = 1e-5     # Sec. 2, after Eq. (1)
GAMMA_DEFAULT = 0.5    # Sec. 3.2
Q16 = 65536.0          # rotation-entry quantum (reading: fixed-point coordinates)

__all__ = [
    "EPS_DEFAULT", "GAMMA_DEFAULT", "quantize_rotation", "gradient", "ngf", "erode_mask",
    "rotate_resample", "fixed_fields", "moving_fields", "correlation_maps_fft",
    "correlation_maps_direct", "similarity_at", "normalise", "argmax_map", "evaluate",
    "RotationResult", "Fields",
]


# ----------------------------------------------------------------------------- rotation
def quantize_rotation(R) -> np.ndarray:
    """Round every entry to the nearest multiple of 2^-16, ties to even (numpy's rint)."""
    R = np.asarray(R, dtype=np.float64)
    return np.rint(R * Q16) / Q16


# ----------------------------------------------------------------------------- NGF, Eq. (1)
def gradient(vol: np.ndarray) -> np.ndarray:
    """Central-difference gradient (g_x, g_y, g_z), unit spacing; zero on the grid border."""
    v = np.asarray(vol, dtype=np.float64)
    g = np.zeros((3,) + v.shape, dtype=np.float64)
    # axis 2 is x, axis 1 is y, axis 0 is z
    g[0][:, :, 1:-1] = (v[:, :, 2:] - v[:, :, :-2]) / 2.0
    g[1][:, 1:-1, :] = (v[:, 2:, :] - v[:, :-2, :]) / 2.0
    g[2][1:-1, :, :] = (v[2:, :, :] - v[:-2, :, :]) / 2.0
    return g


def ngf(vol: np.ndarray, eps: float = EPS_DEFAULT) -> np.ndarray:
    """Eq. (1): grad / sqrt(|grad|^2 + eps^2), shape (3, nz, ny, nx)."""
    g = gradient(vol)
    denom = np.sqrt(np.sum(g * g, axis=0) + eps * eps)
    return g / denom


def erode_mask(m: np.ndarray) -> np.ndarray:
    """m(x) and m(x +- e_k) for every axis k; voxels on the grid border are 0."""
    m = np.asarray(m, dtype=bool)
    out = np.zeros_like(m)
    c = m[1:-1, 1:-1, 1:-1].copy()
    c &= m[1:-1, 1:-1, 2:] & m[1:-1, 1:-1, :-2]
    c &= m[1:-1, 2:, 1:-1] & m[1:-1, :-2, 1:-1]
    c &= m[2:, 1:-1, 1:-1] & m[:-2, 1:-1, 1:-1]
    out[1:-1, 1:-1, 1:-1] = c
    return out


# ----------------------------------------------------------------------------- resample
def rotate_resample(B: np.ndarray, R, mask_b: np.ndarray | None = None):
    """B^ = B o T_R by trilinear interpolation (Sec. 3.2), on B's own grid.

    ``R`` must already be quantised.  Returns (B^, V) where V marks output voxels whose
    source point lies inside B's closed box (and, with a user mask, whose 8 source-cell
    corners are all inside the mask).  B^ is 0 where V is false.
    """
    B = np.asarray(B, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    nz, ny, nx = B.shape
    n = np.array([nx, ny, nz], dtype=np.float64)
    c = (n - 1.0) / 2.0
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([x, y, z], axis=-1).astype(np.float64)
    p = (X - c) @ R.T + c                                   # exact for quantised R
    V = np.all((p >= 0.0) & (p <= n - 1.0), axis=-1)
    i0 = np.floor(p)
    i0 = np.clip(i0, 0.0, n - 2.0)                          # upper edge: weight 1 on n-1
    f = p - i0
    i0 = np.where(V[..., None], i0, 0.0).astype(np.int64)
    f = np.where(V[..., None], f, 0.0)
    ix, iy, iz = i0[..., 0], i0[..., 1], i0[..., 2]
    fx, fy, fz = f[..., 0], f[..., 1], f[..., 2]
    out = np.zeros(B.shape, dtype=np.float64)
    inside = np.ones(B.shape, dtype=bool)
    for dz in (0, 1):
        wz = fz if dz else 1.0 - fz
        for dy in (0, 1):
            wy = fy if dy else 1.0 - fy
            for dx in (0, 1):
                wx = fx if dx else 1.0 - fx
                out += wz * wy * wx * B[iz + dz, iy + dy, ix + dx]
                if mask_b is not None:
                    inside &= np.asarray(mask_b, dtype=bool)[iz + dz, iy + dy, ix + dx]
    if mask_b is not None:
        V = V & inside
    out[~V] = 0.0
    return out, V


# ----------------------------------------------------------------------------- fields
@dataclass
class Fields:
    n: np.ndarray       # (3, nz, ny, nx) NGF
    mask: np.ndarray    # (nz, ny, nx) bool, eroded


def fixed_fields(A, mask_a=None, eps: float = EPS_DEFAULT) -> Fields:
    """NGF and eroded mask of the fixed volume (no rotation)."""
    A = np.asarray(A, dtype=np.float64)
    m = np.ones(A.shape, dtype=bool) if mask_a is None else np.asarray(mask_a, dtype=bool)
    return Fields(ngf(A, eps), erode_mask(m))


def moving_fields(B, R, mask_b=None, eps: float = EPS_DEFAULT) -> Fields:
    """NGF of the rotated-and-resampled moving volume and its eroded validity mask."""
    Bh, V = rotate_resample(B, R, mask_b)
    return Fields(ngf(Bh, eps), erode_mask(V))


# ----------------------------------------------------------------------------- Eq. (5), one chi
def _overlap_slices(shape_a, shape_b, chi_xyz):
    """Slices of A and of B such that A[sa] pairs with B[sb] under x -> x + chi."""
    sa, sb = [], []
    for axis, c in zip((0, 1, 2), (chi_xyz[2], chi_xyz[1], chi_xyz[0])):
        na, nb = shape_a[axis], shape_b[axis]
        lo = max(0, -c)
        hi = min(na, nb - c)
        if hi <= lo:
            return None
        sa.append(slice(lo, hi))
        sb.append(slice(lo + c, hi + c))
    return tuple(sa), tuple(sb)


def similarity_at(fa: Fields, fb: Fields, chi_xyz, measure: str = "squared"):
    """Eq. (5) at a single displacement by direct summation: returns (S, N).

    S = sum_x M_A(x) M_B(x + chi) s(x) with s = <n_A(x), n_B(x + chi)>^2 (Eq. (2)) or, for
    measure="unsquared", s = <n_A(x), n_B(x + chi)> (Eq. (3)); N = sum_x M_A(x) M_B(x + chi).
    """
    sl = _overlap_slices(fa.mask.shape, fb.mask.shape, chi_xyz)
    if sl is None:
        return 0.0, 0
    sa, sb = sl
    m = fa.mask[sa] & fb.mask[sb]
    dot = np.zeros(m.shape, dtype=np.float64)
    for k in range(3):
        dot += fa.n[k][sa] * fb.n[k][sb]
    s = dot if measure == "unsquared" else dot * dot
    return float(np.sum(np.where(m, s, 0.0))), int(np.count_nonzero(m))


def correlation_maps_direct(fa: Fields, fb: Fields, measure: str = "squared"):
    """Eq. (5) numerators and overlaps for every chi by direct summation (small volumes)."""
    nza, nya, nxa = fa.mask.shape
    nzb, nyb, nxb = fb.mask.shape
    W = (nza + nzb - 1, nya + nyb - 1, nxa + nxb - 1)
    S = np.zeros(W, dtype=np.float64)
    N = np.zeros(W, dtype=np.int64)
    for iz in range(W[0]):
        for iy in range(W[1]):
            for ix in range(W[2]):
                chi = (ix - (nxa - 1), iy - (nya - 1), iz - (nza - 1))
                S[iz, iy, ix], N[iz, iy, ix] = similarity_at(fa, fb, chi, measure)
    return S, N


# ----------------------------------------------------------------------------- Eq. (6)-(8)
_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
_WEIGHTS = (1.0, 1.0, 1.0, 2.0, 2.0, 2.0)


def _separable_parts(fa: Fields, fb: Fields, measure: str):
    """(weight, A-side field, B-side field) of the separable expansion: the 6 products of
    Eq. (6) for the squared measure, the 3 components of Eq. (3) for the unsquared one."""
    ma = fa.mask.astype(np.float64)
    mb = fb.mask.astype(np.float64)
    if measure == "unsquared":
        return [(1.0, ma * fa.n[k], mb * fb.n[k]) for k in range(3)]
    if measure != "squared":
        raise ValueError(f"unknown measure {measure!r}")
    return [(w, ma * fa.n[k] * fa.n[l], mb * fb.n[k] * fb.n[l]) for (k, l), w in zip(_PAIRS, _WEIGHTS)]


def _linear_from_circular(circ: np.ndarray, shape_a, shape_b, P_zyx):
    """Pick the linear-correlation displacements out of a circular correlation of size P."""
    idx = []
    for axis in range(3):
        na, nb, p = shape_a[axis], shape_b[axis], P_zyx[axis]
        chi = np.arange(na + nb - 1) - (na - 1)
        idx.append(np.mod(chi, p))
    return circ[np.ix_(*idx)]


def correlation_maps_fft(fa: Fields, fb: Fields, P_xyz=None, measure: str = "squared"):
    """S and N for every chi via zero-padded FP64 FFT cross-correlation (Eq. (6)-(8)).

    S is the sum over the separable parts (6 products with cross products weighted 2, or
    the 3 components for measure="unsquared"), correlated in the frequency domain and
    summed before one inverse transform; N is the mask correlation, rounded to the nearest
    integer (asserting it is within 1e-6 of one).  ``P_xyz`` (each >= n_A + n_B - 1)
    defaults to the smallest size that avoids wrap-around.
    """
    sa, sb = fa.mask.shape, fb.mask.shape
    need = tuple(sa[a] + sb[a] - 1 for a in range(3))
    if P_xyz is None:
        P = need
    else:
        P = (int(P_xyz[2]), int(P_xyz[1]), int(P_xyz[0]))
        if any(P[a] < need[a] for a in range(3)):
            raise ValueError(f"FFT size {P_xyz} smaller than n_A + n_B - 1")
    ma = fa.mask.astype(np.float64)
    mb = fb.mask.astype(np.float64)
    acc = None
    for w, a, b in _separable_parts(fa, fb, measure):
        term = w * np.conj(sfft.rfftn(a, s=P, workers=WORKERS)) * sfft.rfftn(b, s=P, workers=WORKERS)
        acc = term if acc is None else acc + term
    S_circ = sfft.irfftn(acc, s=P, workers=WORKERS)
    N_prod = np.conj(sfft.rfftn(ma, s=P, workers=WORKERS)) * sfft.rfftn(mb, s=P, workers=WORKERS)
    N_circ = sfft.irfftn(N_prod, s=P, workers=WORKERS)
    S = _linear_from_circular(S_circ, sa, sb, P)
    Nf = _linear_from_circular(N_circ, sa, sb, P)
    N = np.rint(Nf)
    resid = float(np.max(np.abs(Nf - N))) if N.size else 0.0
    assert resid < 1e-6, f"overlap count not integral (residual {resid})"
    return S, N.astype(np.int64)


# ----------------------------------------------------------------------------- normalise + argmax
def normalise(S, N, count_a: int, count_b: int, gamma: float = GAMMA_DEFAULT):
    """C = S / N on valid chi (N >= 1 and N >= gamma * min(|M_A|, |M_B^|)), -inf elsewhere."""
    thr = float(gamma) * float(min(count_a, count_b))
    valid = (N >= 1) & (N.astype(np.float64) >= thr)
    C = np.full(S.shape, -np.inf, dtype=np.float64)
    C[valid] = S[valid] / N[valid]
    return C, valid


def argmax_map(C: np.ndarray):
    """Largest C; ties go to the smallest flat (canonical) index.  Returns (score, flat) or None."""
    if not np.any(np.isfinite(C)):
        return None
    flat = int(np.argmax(C))       # numpy returns the first maximal index
    return float(C.flat[flat]), flat


@dataclass
class RotationResult:
    score: float                 # -inf when no chi is valid
    shift: tuple                 # (chi_x, chi_y, chi_z)
    overlap: int
    valid: bool
    R_used: np.ndarray           # quantised matrix
    S: np.ndarray | None = None
    N: np.ndarray | None = None
    C: np.ndarray | None = None


def evaluate(A, B, rotations, mask_a=None, mask_b=None, eps: float = EPS_DEFAULT,
             gamma: float = GAMMA_DEFAULT, P_xyz=None, keep_maps: bool = False,
             method: str = "fft", measure: str = "squared"):
    """Score every rotation over all displacements; return (per-rotation results, best index).

    ``method`` is "fft" (Eq. (6)-(8)) or "direct" (Eq. (5) summed directly; small volumes);
    ``measure`` is "squared" (Eq. (2), CSNGF) or "unsquared" (Eq. (3), USNGF).
    The best index is None when no rotation has a valid displacement.
    """
    fa = fixed_fields(A, mask_a, eps)
    count_a = int(np.count_nonzero(fa.mask))
    nza, nya, nxa = fa.mask.shape
    results = []
    best = None
    for r_idx, R in enumerate(np.asarray(rotations, dtype=np.float64).reshape(-1, 3, 3)):
        Rq = quantize_rotation(R)
        fb = moving_fields(B, Rq, mask_b, eps)
        count_b = int(np.count_nonzero(fb.mask))
        if method == "direct":
            S, N = correlation_maps_direct(fa, fb, measure)
        else:
            S, N = correlation_maps_fft(fa, fb, P_xyz, measure)
        C, _ = normalise(S, N, count_a, count_b, gamma)
        am = argmax_map(C)
        if am is None:
            res = RotationResult(-np.inf, (0, 0, 0), 0, False, Rq)
        else:
            score, flat = am
            iz, iy, ix = np.unravel_index(flat, C.shape)
            shift = (int(ix) - (nxa - 1), int(iy) - (nya - 1), int(iz) - (nza - 1))
            res = RotationResult(score, shift, int(N[iz, iy, ix]), True, Rq)
            if best is None or score > results[best].score:
                best = r_idx
        if keep_maps:
            res.S, res.N, res.C = S, N, C
        results.append(res)
    return results, best
