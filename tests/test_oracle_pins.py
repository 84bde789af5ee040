"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a brute-force loop over
displacements (the direct algorithm of Sec. 5.2), closed forms (orthogonal and parallel
gradient fields, Sec. 2 after Eq. (2)), exact voxel permutations, recovery of a known
integer shift, overlap counts of boxes, and invariances.  Together they make a dropped
term, a wrong weight, sign, index, centre, padding or normalisation fail at least one test.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2110_10156_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_rot(rng, max_deg=40.0):
    return synth.axis_angle_matrix(rng.normal(size=3), math.radians(rng.uniform(0, max_deg)))


# ----------------------------------------------------------------------------- paper constants
def test_paper_constants_match_golden():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        g = json.load(f)
    assert O.EPS_DEFAULT == g["eps"]["value"]
    assert O.GAMMA_DEFAULT == g["gamma"]["value"]


def _ramp(shape_zyx, direction_xyz, beta, offset=0.0):
    nz, ny, nx = shape_zyx
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.asarray(direction_xyz, dtype=np.float64)
    return beta * (d[0] * x + d[1] * y + d[2] * z) + offset


def test_special_values_parallel_antiparallel_orthogonal():
    """Sec. 2: s -> 1 for parallel and anti-parallel gradients, 0 for orthogonal ones."""
    shape = (7, 8, 9)
    A = _ramp(shape, (1, 0, 0), 1.0)
    for B, expect in ((_ramp(shape, (1, 0, 0), 3.0, 2.0), 1.0),
                      (_ramp(shape, (-1, 0, 0), 0.5), 1.0),
                      (_ramp(shape, (0, 1, 0), 1.0), 0.0)):
        res, best = O.evaluate(A, B, np.eye(3)[None], keep_maps=True)
        C = res[0].C
        v = np.isfinite(C)
        assert v.any()
        assert np.max(np.abs(C[v] - expect)) < 1e-9


# ----------------------------------------------------------------------------- quantisation
def test_quantize_rotation_half_even_and_grid():
    q = 1.0 / 65536.0
    R = np.array([[0.5 * q, 1.5 * q, 2.5 * q], [-0.5 * q, -1.5 * q, 1.0], [0.3, -0.7, 1e-9]])
    Rq = O.quantize_rotation(R)
    assert Rq[0, 0] == 0.0 and Rq[0, 1] == 2 * q and Rq[0, 2] == 2 * q
    assert Rq[1, 0] == 0.0 and Rq[1, 1] == -2 * q and Rq[1, 2] == 1.0
    assert np.all(np.abs(Rq * 65536 - np.round(Rq * 65536)) == 0)
    assert np.max(np.abs(Rq - R)) <= 0.5 * q


# ----------------------------------------------------------------------------- NGF, Eq. (1)
def test_ngf_of_ramp_closed_form():
    """A ramp of slope beta has central-difference gradient beta: n = beta / sqrt(beta^2+eps^2)."""
    eps = 1e-5
    for beta in (1e-5, 3e-5, 0.2):
        A = _ramp((5, 6, 7), (0, 0, 1), beta)  # along z
        n = O.ngf(A, eps)
        inner = (slice(1, -1),) * 3
        assert np.allclose(n[2][inner], beta / math.sqrt(beta * beta + eps * eps), rtol=1e-9)
        assert np.all(n[0][inner] == 0) and np.all(n[1][inner] == 0)


def test_mask_erosion_box_and_hole():
    m = np.ones((5, 6, 7), dtype=bool)
    e = O.erode_mask(m)
    assert e.sum() == 3 * 4 * 5 and e[1:-1, 1:-1, 1:-1].all()
    m[2, 3, 3] = False
    e = O.erode_mask(m)
    for dz, dy, dx in ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        assert not e[2 + dz, 3 + dy, 3 + dx]
    assert e.sum() == 3 * 4 * 5 - 7


# ----------------------------------------------------------------------------- resampling
def test_identity_resample_is_bit_exact():
    rng = np.random.default_rng(3)
    B = rng.random((5, 6, 7))
    Bh, V = O.rotate_resample(B, np.eye(3))
    assert V.all() and np.array_equal(Bh, B)


def test_quarter_turn_is_voxel_permutation():
    """90 deg about z on a square cross-section: p = (n-1-y, x, z), an exact permutation."""
    rng = np.random.default_rng(4)
    B = rng.random((5, 8, 8))
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    Bh, V = O.rotate_resample(B, Rz)
    assert V.all()
    expect = np.empty_like(B)
    for z in range(5):
        for y in range(8):
            for x in range(8):
                expect[z, y, x] = B[z, x, 7 - y]
    assert np.array_equal(Bh, expect)
    # 180 deg about x on a cross-section ny x nz: p = (x, n_y-1-y, n_z-1-z)
    Rx = np.diag([1.0, -1.0, -1.0])
    Bh, V = O.rotate_resample(B, Rx)
    assert V.all() and np.array_equal(Bh, B[::-1, ::-1, :])


def test_trilinear_reproduces_affine_and_validity_box():
    rng = np.random.default_rng(5)
    shape = (9, 10, 11)
    a = rng.normal(size=3)
    B = _ramp(shape, a, 1.0, 0.25)
    for _ in range(3):
        Rq = O.quantize_rotation(_rand_rot(rng, 70))
        Bh, V = O.rotate_resample(B, Rq)
        nz, ny, nx = shape
        n = np.array([nx, ny, nz], float)
        c = (n - 1) / 2
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    p = Rq @ (np.array([x, y, z], float) - c) + c
                    inside = bool(np.all(p >= 0) and np.all(p <= n - 1))
                    assert inside == bool(V[z, y, x])
                    if inside:
                        assert abs(Bh[z, y, x] - (a @ p + 0.25)) < 1e-11
                    else:
                        assert Bh[z, y, x] == 0.0


def test_user_mask_on_b_requires_all_cell_corners():
    rng = np.random.default_rng(6)
    B = rng.random((6, 6, 6))
    mb = np.ones(B.shape, dtype=bool)
    mb[3, 3, 3] = False
    # a small non-axis rotation: every output voxel whose source cell touches (3,3,3) is cut
    Rq = O.quantize_rotation(_rand_rot(rng, 10))
    _, V0 = O.rotate_resample(B, Rq)
    _, V1 = O.rotate_resample(B, Rq, mb)
    n = np.array([6, 6, 6], float)
    c = (n - 1) / 2
    for z in range(6):
        for y in range(6):
            for x in range(6):
                if not V0[z, y, x]:
                    assert not V1[z, y, x]
                    continue
                p = Rq @ (np.array([x, y, z], float) - c) + c
                i0 = np.clip(np.floor(p), 0, n - 2).astype(int)
                touches = all(i0[k] <= 3 <= i0[k] + 1 for k in range(3))
                assert V1[z, y, x] == (not touches)


# ----------------------------------------------------------------------------- Eq. (5) brute force
def _brute_force_maps(fa, fb):
    """Pure-Python nested loops over displacements and voxels (the direct algorithm).

    Uses the squared dot product as written in Eq. (2)/(5), not the 6-term expansion.
    """
    na = fa.mask.shape
    nb = fb.mask.shape
    ma, mb = fa.mask.tolist(), fb.mask.tolist()
    A0, A1, A2 = (fa.n[k].tolist() for k in range(3))
    B0, B1, B2 = (fb.n[k].tolist() for k in range(3))
    W = tuple(na[i] + nb[i] - 1 for i in range(3))
    S = np.zeros(W)
    N = np.zeros(W, dtype=np.int64)
    for cz in range(-(na[0] - 1), nb[0]):
        for cy in range(-(na[1] - 1), nb[1]):
            for cx in range(-(na[2] - 1), nb[2]):
                s = 0.0
                cnt = 0
                for z in range(na[0]):
                    zb = z + cz
                    if not 0 <= zb < nb[0]:
                        continue
                    for y in range(na[1]):
                        yb = y + cy
                        if not 0 <= yb < nb[1]:
                            continue
                        for x in range(na[2]):
                            xb = x + cx
                            if not 0 <= xb < nb[2]:
                                continue
                            if ma[z][y][x] and mb[zb][yb][xb]:
                                d = (A0[z][y][x] * B0[zb][yb][xb] + A1[z][y][x] * B1[zb][yb][xb]
                                     + A2[z][y][x] * B2[zb][yb][xb])
                                s += d * d
                                cnt += 1
                idx = (cz + na[0] - 1, cy + na[1] - 1, cx + na[2] - 1)
                S[idx] = s
                N[idx] = cnt
    return S, N


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fft_route_matches_brute_force(seed):
    """P1: Eq. (6)-(8) through zero-padded FFTs equals Eq. (5) summed directly."""
    rng = np.random.default_rng(100 + seed)
    sa = tuple(int(v) for v in rng.integers(4, 7, size=3))
    sb = tuple(int(v) for v in rng.integers(4, 7, size=3))
    A = rng.random(sa)
    B = rng.random(sb)
    ma = rng.random(sa) > 0.15 if seed != 0 else None
    mb = rng.random(sb) > 0.1 if seed == 2 else None
    Rq = O.quantize_rotation(_rand_rot(rng, 25))
    fa = O.fixed_fields(A, ma)
    fb = O.moving_fields(B, Rq, mb)
    Sb, Nb = _brute_force_maps(fa, fb)
    Sf, Nf = O.correlation_maps_fft(fa, fb)
    assert np.array_equal(Nf, Nb)
    assert np.max(np.abs(Sf - Sb)) < 1e-12
    Sd, Nd = O.correlation_maps_direct(fa, fb)
    assert np.array_equal(Nd, Nb) and np.max(np.abs(Sd - Sb)) < 1e-12
    # padding larger than needed and odd sizes change nothing on the linear range (P9)
    big = tuple(sa[2 - i] + sb[2 - i] + int(rng.integers(0, 5)) for i in range(3))
    Sp, Np = O.correlation_maps_fft(fa, fb, P_xyz=big)
    assert np.array_equal(Np, Nb) and np.max(np.abs(Sp - Sb)) < 1e-12


@pytest.mark.parametrize("gamma", [0.25, 0.5])
def test_evaluate_fft_equals_direct_including_gamma_and_argmax(gamma):
    rng = np.random.default_rng(7)
    A = rng.random((6, 5, 7))
    B = rng.random((5, 7, 6))
    rots = np.stack([np.eye(3), _rand_rot(rng), _rand_rot(rng)])
    rf, bf = O.evaluate(A, B, rots, gamma=gamma, keep_maps=True)
    rd, bd = O.evaluate(A, B, rots, gamma=gamma, keep_maps=True, method="direct")
    assert bf == bd
    for a, b in zip(rf, rd):
        assert np.array_equal(np.isfinite(a.C), np.isfinite(b.C))
        v = np.isfinite(a.C)
        assert np.max(np.abs(a.C[v] - b.C[v])) < 1e-12
        assert a.shift == b.shift and a.overlap == b.overlap


# ----------------------------------------------------------------------------- closed forms
def test_orthogonal_fields_give_zero():
    """P2: x-ramp against y-ramp: every product pair has a zero factor, S == 0."""
    shape = (6, 7, 8)
    A = _ramp(shape, (1, 0, 0), 0.3)
    B = _ramp(shape, (0, 1, 0), 0.7, 1.0)
    fa, fb = O.fixed_fields(A), O.moving_fields(B, np.eye(3))
    S, N = O.correlation_maps_fft(fa, fb)
    assert np.max(np.abs(S)) < 1e-12
    for chi in ((0, 0, 0), (2, -1, 1), (-3, 2, 0)):
        s, n = O.similarity_at(fa, fb, chi)
        assert s == 0.0 and n > 0


@pytest.mark.parametrize("case", range(4))
def test_parallel_fields_closed_form_under_rotation(case):
    """P3: A = bA (d.x), B = +-bB (d.x) + o.  After resampling with Rq, grad B^ = +-bB Rq^T d
    exactly (trilinear interpolation reproduces affine functions), so C is the constant
    (n_A . n_B^)^2 with n = g / sqrt(|g|^2 + eps^2) on every valid displacement."""
    rng = np.random.default_rng(20 + case)
    eps = 1e-5
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    bA = [1e-5, 2e-5, 0.3, 1.0][case]       # |g_A| near eps makes eps matter
    bB = [0.5, 1e-5, 3e-5, 2.0][case]
    sign = -1.0 if case % 2 else 1.0
    sa, sb = (9, 8, 10), (8, 10, 9)
    A = _ramp(sa, d, bA)
    B = _ramp(sb, sign * d, bB, 0.5)
    R = np.eye(3) if case == 0 else _rand_rot(rng, 35)
    Rq = O.quantize_rotation(R)
    gA = bA * d
    gB = sign * bB * (Rq.T @ d)
    nA = gA / math.sqrt(gA @ gA + eps * eps)
    nB = gB / math.sqrt(gB @ gB + eps * eps)
    expect = float(nA @ nB) ** 2
    res, _ = O.evaluate(A, B, R[None], eps=eps, keep_maps=True)
    C = res[0].C
    v = np.isfinite(C)
    assert v.sum() > 10
    assert np.max(np.abs(C[v] - expect)) < 1e-9 * max(1.0, expect)


def test_sign_invariance_bit_identical():
    """P4: C(A, -B) == C(A, B) exactly: every product n_k n_l is invariant under n -> -n."""
    rng = np.random.default_rng(8)
    A, B = rng.random((6, 7, 6)), rng.random((7, 6, 6))
    R = _rand_rot(rng)[None]
    r1, _ = O.evaluate(A, B, R, keep_maps=True)
    r2, _ = O.evaluate(A, -B, R, keep_maps=True)
    assert np.array_equal(r1[0].C, r2[0].C) and np.array_equal(r1[0].N, r2[0].N)


def test_swap_symmetry_at_identity():
    """P5: with n_A = n_B and no rotation, C_{A,B}(chi) = C_{B,A}(-chi)."""
    rng = np.random.default_rng(9)
    A, B = rng.random((6, 7, 8)), rng.random((6, 7, 8))
    r1, _ = O.evaluate(A, B, np.eye(3)[None], keep_maps=True)
    r2, _ = O.evaluate(B, A, np.eye(3)[None], keep_maps=True)
    C1, C2 = r1[0].C, r2[0].C[::-1, ::-1, ::-1]
    assert np.array_equal(np.isfinite(C1), np.isfinite(C2))
    v = np.isfinite(C1)
    assert np.max(np.abs(C1[v] - C2[v])) < 1e-12
    assert np.array_equal(r1[0].N, r2[0].N[::-1, ::-1, ::-1])


def test_overlap_closed_form_and_gamma_rule():
    """P7: identity rotation, no user masks: both eroded masks are boxes [1, n-2] and
    N(chi) = prod_k max(0, min(nA_k-2, nB_k-2-chi_k) - max(1, 1-chi_k) + 1)."""
    rng = np.random.default_rng(10)
    sa, sb = (6, 8, 7), (9, 5, 8)        # (z, y, x)
    A, B = rng.random(sa), rng.random(sb)
    for gamma in (0.25, 0.5, 0.75):
        res, _ = O.evaluate(A, B, np.eye(3)[None], gamma=gamma, keep_maps=True)
        N, C = res[0].N, res[0].C
        nA = (sa[2], sa[1], sa[0])
        nB = (sb[2], sb[1], sb[0])
        cnt_a = np.prod([v - 2 for v in nA])
        cnt_b = np.prod([v - 2 for v in nB])
        for iz in range(N.shape[0]):
            for iy in range(N.shape[1]):
                for ix in range(N.shape[2]):
                    chi = (ix - (nA[0] - 1), iy - (nA[1] - 1), iz - (nA[2] - 1))
                    expect = 1
                    for k in range(3):
                        expect *= max(0, min(nA[k] - 2, nB[k] - 2 - chi[k]) - max(1, 1 - chi[k]) + 1)
                    assert N[iz, iy, ix] == expect
                    valid = expect >= 1 and expect >= gamma * min(cnt_a, cnt_b)
                    assert np.isfinite(C[iz, iy, ix]) == valid


def test_range_and_numerator_bound():
    """P10: 0 <= C <= 1 and S <= N on every displacement."""
    rng = np.random.default_rng(11)
    A, B = rng.random((7, 6, 7)), rng.random((6, 7, 7))
    res, _ = O.evaluate(A, B, _rand_rot(rng)[None], gamma=0.0, keep_maps=True)
    S, N, C = res[0].S, res[0].N, res[0].C
    assert np.all(S <= N + 1e-9) and np.all(S >= -1e-9)
    v = np.isfinite(C)
    assert np.all(C[v] >= -1e-12) and np.all(C[v] <= 1 + 1e-12)


@pytest.mark.parametrize("tenths", [1, 3, 7, 9])
def test_gamma_rule_exact_for_decimal_fractions(tenths):
    """Sec. 3.2's minimum overlap N >= gamma * m for gamma = tenths / 10, checked against exact
    rational arithmetic (10 N >= tenths * m) at every N around the threshold, including the
    m for which gamma * m is an integer (validity must hold there: N = gamma * m meets it)."""
    from fractions import Fraction
    gamma = tenths / 10.0
    for m in (10, 20, 30, 70, 1000, 3_000_000, 3_232_110, 7, 13, 333_333):
        lo = max(0, int(tenths * m // 10) - 3)
        N = np.arange(lo, lo + 8, dtype=np.int64)
        S = np.zeros(N.shape)
        for ca, cb in ((m, m + 5), (m + 9, m)):         # m = min(|M_A|, |M_B^|) either way
            _, valid = O.normalise(S, N, ca, cb, gamma)
            exact = (N >= 1) & np.array([Fraction(int(n)) >= Fraction(tenths, 10) * m for n in N])
            assert np.array_equal(valid, exact), (tenths, m, N[valid != exact])


def test_cross_rotation_tie_goes_to_the_smaller_index():
    """Equal best scores across rotations: the smaller rotation index wins.  The same matrix
    twice gives bit-identical maps, so the first copy must be reported, wherever it sits."""
    rng = np.random.default_rng(12)
    A, B = rng.random((7, 8, 6)), rng.random((6, 7, 8))
    R1, R2 = _rand_rot(rng, 30), _rand_rot(rng, 30)
    res, best = O.evaluate(A, B, np.stack([R1, R1]))
    assert res[0].score == res[1].score and best == 0
    res, best = O.evaluate(A, B, np.stack([R2, R1, R1, R2]))
    top = max(r.score for r in res)
    assert best == min(i for i, r in enumerate(res) if r.score == top)
    assert res[0].score == res[3].score and res[1].score == res[2].score
    assert best in (0, 1)


def test_argmax_tie_break_smallest_canonical_index():
    C = np.full((3, 3, 3), -np.inf)
    C[2, 0, 0] = 0.5
    C[0, 2, 1] = 0.5
    C[0, 2, 2] = 0.5
    assert O.argmax_map(C) == (0.5, np.ravel_multi_index((0, 2, 1), C.shape))
    assert O.argmax_map(np.full((2, 2, 2), -np.inf)) is None


# ----------------------------------------------------------------------------- shift recovery
def test_known_integer_shift_is_recovered_config0():
    """P6: B is f(A) translated by t plus noise; the argmax displacement is t."""
    pair = synth.config0()
    res, best = O.evaluate(pair.A, pair.B, pair.rotations)
    assert best == 0
    assert res[0].shift == pair.true_shift


@pytest.mark.parametrize("t", [(3, -2, 5), (-6, 6, 0)])
def test_translated_copy_recovers_shift(t):
    """B(y) = A(y - t) (exact array translation, no intensity change): argmax chi = t."""
    rng = np.random.default_rng(12)
    A = rng.random((20, 22, 24))
    from scipy.ndimage import gaussian_filter
    A = gaussian_filter(A, 1.0)
    B = np.zeros_like(A)
    tx, ty, tz = t
    src = A[max(0, -tz):A.shape[0] - max(0, tz), max(0, -ty):A.shape[1] - max(0, ty),
            max(0, -tx):A.shape[2] - max(0, tx)]
    B[max(0, tz):max(0, tz) + src.shape[0], max(0, ty):max(0, ty) + src.shape[1],
      max(0, tx):max(0, tx) + src.shape[2]] = src
    res, best = O.evaluate(A, B, np.eye(3)[None])
    assert res[0].shift == t


# ----------------------------------------------------------------------------- USNGF, Eq. (3)
def _brute_force_unsquared(fa, fb):
    """Nested loops with the plain (unsquared) dot product of Eq. (3)."""
    na, nb = fa.mask.shape, fb.mask.shape
    ma, mb = fa.mask.tolist(), fb.mask.tolist()
    A = [fa.n[k].tolist() for k in range(3)]
    B = [fb.n[k].tolist() for k in range(3)]
    W = tuple(na[i] + nb[i] - 1 for i in range(3))
    S = np.zeros(W)
    for cz in range(-(na[0] - 1), nb[0]):
        for cy in range(-(na[1] - 1), nb[1]):
            for cx in range(-(na[2] - 1), nb[2]):
                s = 0.0
                for z in range(max(0, -cz), min(na[0], nb[0] - cz)):
                    for y in range(max(0, -cy), min(na[1], nb[1] - cy)):
                        for x in range(max(0, -cx), min(na[2], nb[2] - cx)):
                            if ma[z][y][x] and mb[z + cz][y + cy][x + cx]:
                                s += sum(A[k][z][y][x] * B[k][z + cz][y + cy][x + cx] for k in range(3))
                S[cz + na[0] - 1, cy + na[1] - 1, cx + na[2] - 1] = s
    return S


def test_unsquared_fft_route_matches_brute_force():
    rng = np.random.default_rng(31)
    A, B = rng.random((5, 6, 4)), rng.random((4, 5, 6))
    Rq = O.quantize_rotation(_rand_rot(rng, 30))
    fa, fb = O.fixed_fields(A, rng.random(A.shape) > 0.1), O.moving_fields(B, Rq)
    Sb = _brute_force_unsquared(fa, fb)
    Sf, _ = O.correlation_maps_fft(fa, fb, measure="unsquared")
    Sd, _ = O.correlation_maps_direct(fa, fb, measure="unsquared")
    assert np.max(np.abs(Sf - Sb)) < 1e-12 and np.max(np.abs(Sd - Sb)) < 1e-12


def test_unsquared_is_antisymmetric_in_the_sign_of_b():
    """Eq. (3) changes sign with the gradient sign (the sensitivity Sec. 2 and Sec. 5.1 discuss):
    C_us(A, -B) = -C_us(A, B) exactly, while the squared measure is unchanged."""
    rng = np.random.default_rng(32)
    A, B = rng.random((6, 6, 7)), rng.random((7, 6, 6))
    R = _rand_rot(rng)[None]
    r1, _ = O.evaluate(A, B, R, keep_maps=True, measure="unsquared")
    r2, _ = O.evaluate(A, -B, R, keep_maps=True, measure="unsquared")
    v = np.isfinite(r1[0].C)
    assert np.array_equal(np.isfinite(r2[0].C), v)
    assert np.array_equal(r1[0].C[v], -r2[0].C[v])


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_unsquared_parallel_and_orthogonal_closed_forms(sign):
    rng = np.random.default_rng(33)
    eps = 1e-5
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    A = _ramp((8, 9, 8), d, 2e-5)
    B = _ramp((9, 8, 8), sign * d, 0.4, 0.1)
    R = _rand_rot(rng, 30)
    Rq = O.quantize_rotation(R)
    gA, gB = 2e-5 * d, sign * 0.4 * (Rq.T @ d)
    expect = float((gA / math.sqrt(gA @ gA + eps * eps)) @ (gB / math.sqrt(gB @ gB + eps * eps)))
    res, _ = O.evaluate(A, B, R[None], keep_maps=True, measure="unsquared")
    C = res[0].C
    v = np.isfinite(C)
    assert v.sum() > 10 and np.max(np.abs(C[v] - expect)) < 1e-9
    assert np.sign(expect) == sign
    # squared measure on the same pair is the square of the unsquared one
    rs, _ = O.evaluate(A, B, R[None], keep_maps=True)
    assert np.max(np.abs(rs[0].C[v] - expect ** 2)) < 1e-9
    # orthogonal ramps: zero
    Ao = _ramp((8, 9, 8), (1, 0, 0), 0.3)
    Bo = _ramp((9, 8, 8), (0, 0, 1), 0.3)
    ro, _ = O.evaluate(Ao, Bo, np.eye(3)[None], keep_maps=True, measure="unsquared")
    vo = np.isfinite(ro[0].C)
    assert np.max(np.abs(ro[0].C[vo])) < 1e-12
