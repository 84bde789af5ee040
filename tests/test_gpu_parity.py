"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar: overlap counts N exact, validity sets identical, |C_gpu - C_oracle| <= 1e-4 on valid
displacements (the FP32 tolerance of the hot path), per-rotation argmax identical unless the
oracle's best and runner-up are within 2e-4 (then the GPU's pick must score within 2e-4 of
the oracle's best), and the overall (rotation, displacement) identical.
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
TIE = 2e-4


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _rand_rot(rng, max_deg=40.0):
    return synth.axis_angle_matrix(rng.normal(size=3), math.radians(rng.uniform(0, max_deg)))


def _oracle_maps(A, B, R, mask_b=None, gamma=0.5, P=None, mask_a=None, measure="squared"):
    fa = O.fixed_fields(A, mask_a)
    fb = O.moving_fields(B, O.quantize_rotation(R), mask_b)
    S, N = O.correlation_maps_fft(fa, fb, P, measure=measure)
    C, valid = O.normalise(S, N, int(fa.mask.sum()), int(fb.mask.sum()), gamma)
    return C, N, valid


def _compare_maps(Cg, Ng, Co, No, tag):
    assert Cg.shape == Co.shape, tag
    assert np.array_equal(Ng, No), f"{tag}: overlap counts differ at {np.argwhere(Ng != No)[:5]}"
    vg, vo = np.isfinite(Cg), np.isfinite(Co)
    assert np.array_equal(vg, vo), f"{tag}: validity differs"
    if vo.any():
        err = float(np.max(np.abs(Cg[vo].astype(np.float64) - Co[vo])))
        _say(tag, "max|dC| =", err, "valid =", int(vo.sum()))
        assert err <= CTOL, f"{tag}: max |dC| {err}"
        go, gg = O.argmax_map(Co), int(np.argmax(np.where(vg, Cg, -np.inf)))
        sorted_o = np.sort(Co[vo])[::-1]
        gap = sorted_o[0] - sorted_o[1] if sorted_o.size > 1 else np.inf
        if gap >= TIE:
            assert gg == go[1], f"{tag}: argmax {gg} vs {go[1]}"
        else:
            assert Co.flat[gg] >= go[0] - TIE


# ----------------------------------------------------------------------------- FFT engine
FFT_LENGTHS = [8, 10, 12, 14, 16, 20, 22, 24, 28, 32, 40, 44, 48, 56, 64, 66, 88, 96, 110, 112, 128, 160, 176,
               192, 198, 220, 240, 256, 264, 320, 330, 352, 384, 440, 448, 480, 512]


@pytest.mark.parametrize("inverse", [False, True])
def test_fft_engine_against_numpy(inverse):
    import torch
    rng = np.random.default_rng(1)
    for L in FFT_LENGTHS:
        _say("fft", L, "inverse" if inverse else "forward")
        batch = 37
        x = (rng.normal(size=(batch, L)) + 1j * rng.normal(size=(batch, L))).astype(np.complex64)
        xd = torch.from_numpy(x).cuda()
        yd = torch.empty_like(xd)
        bd.debug_fft(xd, inverse=inverse, out=yd)
        y = yd.cpu().numpy().astype(np.complex128)
        ref = np.fft.ifft(x.astype(np.complex128), axis=1) * L if inverse else np.fft.fft(x.astype(np.complex128), axis=1)
        # FP32 FFT bound: error ~ c * 2^-24 * log2(L) * ||x||_2 per row
        norm = np.sqrt(np.sum(np.abs(x) ** 2, axis=1, keepdims=True))
        err = np.max(np.abs(y - ref) / norm)
        assert err < 4 * 2.0 ** -24 * math.log2(L), (L, err)
    # delta -> constant, constant -> delta
    for L in (64, 220, 352):
        d = np.zeros((16, L), np.complex64)
        d[:, 0] = 1
        yd = bd.debug_fft(torch.from_numpy(d).cuda(), inverse=inverse).cpu().numpy()
        assert np.max(np.abs(yd - 1)) < 1e-6
        c = np.ones((16, L), np.complex64)
        yc = bd.debug_fft(torch.from_numpy(c).cuda(), inverse=inverse).cpu().numpy()
        e = np.zeros(L)
        e[0] = L
        assert np.max(np.abs(yc - e)) < 1e-4 * L


# ----------------------------------------------------------------------------- field stage
def _field_bound(vol, n_oracle_g, eps):
    """Per-voxel error budget of FP32 products: resampled values carry a few ulps of |B|,
    which the NGF divides by sqrt(|g|^2 + eps^2)."""
    scale = float(np.max(np.abs(vol)))
    return 1e-6 + 16 * 2.0 ** -24 * scale / np.sqrt(n_oracle_g + eps * eps)


@pytest.mark.parametrize("which", ["fixed", "fixed-masked", "identity", "rotated", "masked"])
def test_field_stage_against_oracle(which):
    rng = np.random.default_rng(2)
    pair = synth.config0()
    eps = 1e-5
    fixed = which.startswith("fixed")
    vol = pair.A if fixed else pair.B
    R = None if fixed else (np.eye(3) if which == "identity" else _rand_rot(rng, 50))
    mask = None
    if which in ("masked", "fixed-masked"):
        mask = (rng.random(vol.shape) > 0.02).astype(np.uint8)
    _say("fields", which)
    prod, m = bd.debug_fields(vol, R=R, mask=mask, eps=eps)
    if R is None:
        f = O.fixed_fields(vol, None if mask is None else mask.astype(bool), eps)
        g = O.gradient(vol)
    else:
        Rq = O.quantize_rotation(R)
        f = O.moving_fields(vol, Rq, None if mask is None else mask.astype(bool), eps)
        Bh, _ = O.rotate_resample(vol, Rq, None if mask is None else mask.astype(bool))
        g = O.gradient(Bh)
    assert np.array_equal(m.astype(bool), f.mask), "eroded masks differ"
    g2 = np.sum(g * g, axis=0)
    bound = _field_bound(vol, g2, eps)
    for i, (k, l) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        ref = np.where(f.mask, f.n[k] * f.n[l], 0.0)
        err = np.abs(prod[i] - ref)
        assert np.all(err <= bound), (which, i, float(np.max(err - bound)))


# ----------------------------------------------------------------------------- full maps
def test_config0_maps_and_shift_recovery():
    pair = synth.config0()
    _say("config0 map")
    with bd.Context(pair.A, pair.dims_b, pad=pair.pad) as ctx:
        assert tuple(ctx.info().pad) == (64, 64, 64)
        Cg, Ng = ctx.evaluate_map(pair.B, np.eye(3))
        per, best = ctx.evaluate(pair.B, pair.rotations)
    Co, No, _ = _oracle_maps(pair.A, pair.B, np.eye(3), P=pair.pad)
    _compare_maps(Cg, Ng, Co, No, "config0")
    assert best.rot_index == 0 and tuple(best.shift) == pair.true_shift
    res, _ = O.evaluate(pair.A, pair.B, pair.rotations, P_xyz=pair.pad)
    assert tuple(per[0].shift) == res[0].shift and per[0].overlap == res[0].overlap
    assert abs(per[0].score - res[0].score) <= CTOL


@pytest.mark.parametrize("case", range(6))
def test_random_small_pairs_full_maps(case):
    """Uneven shapes (ragged tiles), n_A != n_B, rotations, user masks on B, gamma 0.25/0.5,
    automatic and explicit padding."""
    rng = np.random.default_rng(50 + case)
    sa = tuple(int(v) for v in rng.integers(5, 23, size=3))
    sb = tuple(int(v) for v in rng.integers(5, 23, size=3))
    from scipy.ndimage import gaussian_filter
    A = gaussian_filter(rng.random(sa), 1.0).astype(np.float32)
    B = gaussian_filter(rng.random(sb), 1.0).astype(np.float32)
    gamma = (0.25, 0.5)[case % 2]
    mask_b = (rng.random(sb) > 0.03).astype(np.uint8) if case >= 3 else None
    R = np.eye(3) if case == 0 else _rand_rot(rng, 60)
    _say("random", case, sa, sb, gamma, mask_b is not None)
    pad = (0, 0, 0)
    if case == 5:  # explicit padding well above n_A + n_B - 1
        need = [sa[2] + sb[2] - 1, sa[1] + sb[1] - 1, sa[0] + sb[0] - 1]
        pad = tuple(next(L for L in range(n + 7, 513) if bd.supported_length(L)) for n in need)
    with bd.Context(A, bd.dims_of(B), gamma=gamma, pad=pad) as ctx:
        P = tuple(ctx.info().pad)
        Cg, Ng = ctx.evaluate_map(B, R, mask_b=mask_b)
        per, best = ctx.evaluate(B, np.stack([R, np.eye(3)]), mask_b=mask_b)
    Co, No, _ = _oracle_maps(A, B, R, None if mask_b is None else mask_b.astype(bool), gamma, P)
    _compare_maps(Cg, Ng, Co, No, f"random{case}")
    # the per-rotation result of evaluate() equals the map's argmax
    if np.isfinite(Cg).any():
        flat = int(np.argmax(np.where(np.isfinite(Cg), Cg, -np.inf)))
        iz, iy, ix = np.unravel_index(flat, Cg.shape)
        assert tuple(per[0].shift) == (ix - (sa[2] - 1), iy - (sa[1] - 1), iz - (sa[0] - 1))
        assert per[0].score == Cg.flat[flat] and per[0].overlap == Ng.flat[flat]


@pytest.mark.parametrize("sa,sb,pz", [((20, 18, 40), (22, 17, 38), 88), ((24, 20, 30), (21, 23, 50), 88),
                                      ((24, 20, 40), (21, 23, 50), 110), ((16, 16, 30), (16, 16, 30), 176)])
def test_compile_time_z_plans_with_radix_11_first(sa, sb, pz):
    """z lengths whose compile-time plan starts with radix 11 (88, 110, 176, like the
    paper-scale 220), with B's interior z extent at most half the length (first stage pruned to
    6 inputs) and above it (the second case: 48 > 44, all 11 inputs), ragged x and y tiles; one
    rotated map and the per-rotation result against the oracle."""
    rng = np.random.default_rng(pz + sa[0])
    from scipy.ndimage import gaussian_filter
    shape_a, shape_b = sa[::-1], sb[::-1]    # (z, y, x) arrays of x, y, z extents
    A = gaussian_filter(rng.random(shape_a), 1.0).astype(np.float32)
    B = gaussian_filter(rng.random(shape_b), 1.0).astype(np.float32)
    R = _rand_rot(rng, 35)
    need = [sa[i] + sb[i] - 1 for i in range(3)]
    assert need[2] <= pz
    pad = (0, 0, pz)
    with bd.Context(A, bd.dims_of(B), pad=pad) as ctx:
        P = tuple(ctx.info().pad)
        assert P[2] == pz
        Cg, Ng = ctx.evaluate_map(B, R)
        per, best = ctx.evaluate(B, np.stack([R, np.eye(3)]))
    _say("radix-11 z plan", sa, sb, P)
    Co, No, _ = _oracle_maps(A, B, R, None, 0.5, P)
    _compare_maps(Cg, Ng, Co, No, f"z{pz}")
    if np.isfinite(Cg).any():
        flat = int(np.argmax(np.where(np.isfinite(Cg), Cg, -np.inf)))
        iz, iy, ix = np.unravel_index(flat, Cg.shape)
        assert tuple(per[0].shift) == (ix - (sa[0] - 1), iy - (sa[1] - 1), iz - (sa[2] - 1))


def test_large_xy_extent_full_maps():
    """A 256 x 256 cross-section: FFT length 512 along x and y (the largest supported; run-time
    plans), slice prefix sums above 16 bits, and the field stage's widest rows."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(77)
    sa, sb = (4, 256, 256), (5, 256, 256)   # (nz, ny, nx)
    A = gaussian_filter(rng.random(sa), 1.5).astype(np.float32)
    B = gaussian_filter(rng.random(sb), 1.5).astype(np.float32)
    R = synth.axis_angle_matrix(np.array([0.0, 0.0, 1.0]), math.radians(20.0))   # in-plane: the thin slab stays valid
    _say("large xy extent", sa, sb)
    with bd.Context(A, bd.dims_of(B)) as ctx:
        P = tuple(ctx.info().pad)
        assert P[0] == 512 and P[1] == 512
        Cg, Ng = ctx.evaluate_map(B, R)
    Co, No, _ = _oracle_maps(A, B, R, None, 0.5, P)
    _compare_maps(Cg, Ng, Co, No, "large-xy")


def _mask_of_a(rng, shape, kind):
    """A user mask on the fixed volume (Sec. 3.1: masks select sub-regions)."""
    nz, ny, nx = shape
    if kind == "random":
        return (rng.random(shape) > 0.1).astype(np.uint8)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = [(n - 1) / 2 for n in shape]
    r = ((z - c[0]) / (0.5 * nz)) ** 2 + ((y - c[1]) / (0.5 * ny)) ** 2 + ((x - c[2]) / (0.45 * nx)) ** 2
    m = r <= 1.0
    if kind == "ellipsoid-holes":
        m &= rng.random(shape) > 0.05
    if kind == "two-blocks":   # a mask in two separate pieces, so its bounding box is not its shape
        m = np.zeros(shape, bool)
        m[:, : ny // 2, : nx // 2] = True
        m[nz // 3:, ny // 2 + 1:, nx // 2 + 1:] = True
    return m.astype(np.uint8)


@pytest.mark.parametrize("case", range(7))
def test_user_mask_on_fixed_volume_full_maps(case):
    """Sec. 3.1, Eq. (4)-(5) with a user mask on A: N(chi) is then the mask cross-correlation,
    computed by the FP64 overlap chain and rounded.  N exact, validity identical, |dC| <= 1e-4,
    over whole maps: random, ellipsoidal, holed and two-piece masks, masks on both volumes,
    gamma 0.25 / 0.5 / 0.3, the unsquared measure, explicit padding, n_A != n_B."""
    rng = np.random.default_rng(300 + case)
    from scipy.ndimage import gaussian_filter
    sa = tuple(int(v) for v in rng.integers(6, 23, size=3))
    sb = tuple(int(v) for v in rng.integers(6, 23, size=3))
    A = gaussian_filter(rng.random(sa), 1.0).astype(np.float32)
    B = gaussian_filter(rng.random(sb), 1.0).astype(np.float32)
    kind = ("random", "ellipsoid", "ellipsoid-holes", "two-blocks", "random", "ellipsoid-holes", "random")[case]
    mask_a = _mask_of_a(rng, sa, kind)
    mask_b = (rng.random(sb) > 0.03).astype(np.uint8) if case in (3, 5) else None
    gamma = (0.5, 0.25, 0.5, 0.3, 0.25, 0.25, 0.5)[case]
    measure = "unsquared" if case == 4 else "squared"
    R = np.eye(3) if case == 0 else _rand_rot(rng, 60)
    pad = (0, 0, 0)
    if case == 6:  # explicit padding above n_A + n_B - 1
        need = [sa[2] + sb[2] - 1, sa[1] + sb[1] - 1, sa[0] + sb[0] - 1]
        pad = tuple(next(L for L in range(n + 5, 513) if bd.supported_length(L)) for n in need)
    _say("mask on A", case, kind, sa, sb, gamma, measure, mask_b is not None)
    with bd.Context(A, bd.dims_of(B), mask_a=mask_a, gamma=gamma, pad=pad, measure=measure) as ctx:
        P = tuple(ctx.info().pad)
        assert ctx.info().count_a == int(O.fixed_fields(A, mask_a.astype(bool)).mask.sum())
        Cg, Ng = ctx.evaluate_map(B, R, mask_b=mask_b)
        per, best = ctx.evaluate(B, np.stack([R, np.eye(3)]), mask_b=mask_b)
    Co, No, _ = _oracle_maps(A, B, R, None if mask_b is None else mask_b.astype(bool), gamma, P,
                             mask_a=mask_a.astype(bool), measure=measure)
    _compare_maps(Cg, Ng, Co, No, f"maskA{case}")
    if np.isfinite(Cg).any():
        flat = int(np.argmax(np.where(np.isfinite(Cg), Cg, -np.inf)))
        iz, iy, ix = np.unravel_index(flat, Cg.shape)
        assert tuple(per[0].shift) == (ix - (sa[2] - 1), iy - (sa[1] - 1), iz - (sa[0] - 1))
        assert per[0].score == Cg.flat[flat] and per[0].overlap == Ng.flat[flat]


def test_all_ones_mask_on_a_equals_no_mask_and_empty_mask_has_no_shift():
    """A mask of ones erodes to the same box as no mask: the FP64 overlap chain must give the
    SAT box sums' counts, so maps and results are bit-identical.  An empty mask leaves no
    valid displacement."""
    pair = synth.config0()
    rng = np.random.default_rng(8)
    rots = np.stack([np.eye(3), _rand_rot(rng, 40), _rand_rot(rng, 40)])
    with bd.Context(pair.A, pair.dims_b) as c0, \
            bd.Context(pair.A, pair.dims_b, mask_a=np.ones(pair.A.shape, np.uint8)) as c1:
        assert c0.info().count_a == c1.info().count_a
        p0, b0 = c0.evaluate(pair.B, rots)
        p1, b1 = c1.evaluate(pair.B, rots)
        C0, N0 = c0.evaluate_map(pair.B, rots[1])
        C1, N1 = c1.evaluate_map(pair.B, rots[1])
    assert np.array_equal(N0, N1) and np.array_equal(C0, C1)
    for a, b in zip(p0, p1):
        assert a.score == b.score and tuple(a.shift) == tuple(b.shift) and a.overlap == b.overlap
    assert b0.rot_index == b1.rot_index == 0
    with bd.Context(pair.A, pair.dims_b, mask_a=np.zeros(pair.A.shape, np.uint8)) as ce:
        assert ce.info().count_a == 0
        per, best = ce.evaluate(pair.B, rots)
        Ce, Ne = ce.evaluate_map(pair.B, rots[0])
    assert best.rot_index == -1 and not any(p.valid for p in per)
    assert not np.isfinite(Ce).any() and not Ne.any()


@pytest.mark.parametrize("seed", [107, 115, 119])
def test_gamma_zero_small_overlaps(seed):
    """gamma = 0 admits every displacement with N >= 1.  On the FP32 path S comes from an FP32
    FFT whose absolute error follows the fields' energy, and C = S / N passes it on undivided
    where N is tiny, so the 1e-4 bar is checked where N >= 10; below that the absolute error of S
    (= dC * N) is bounded instead.  N and validity are exact everywhere.  (The FP64 correlation,
    CSNGF_FP64, meets 1e-4 at every overlap of these pairs: the next test.)"""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    sa = tuple(int(v) for v in rng.integers(3, 30, size=3))
    sb = tuple(int(v) for v in rng.integers(3, 30, size=3))
    A = gaussian_filter(rng.random(sa), 1.0).astype(np.float32)
    B = gaussian_filter(rng.random(sb), 1.0).astype(np.float32)
    R = _rand_rot(rng, 60)
    _say("gamma 0", seed, sa, sb)
    with bd.Context(A, bd.dims_of(B), gamma=0.0) as ctx:
        P = tuple(ctx.info().pad)
        Cg, Ng = ctx.evaluate_map(B, R)
    Co, No, _ = _oracle_maps(A, B, R, None, 0.0, P)
    assert np.array_equal(Ng, No)
    vg, vo = np.isfinite(Cg), np.isfinite(Co)
    assert np.array_equal(vg, vo)
    d = np.abs(Cg[vo].astype(np.float64) - Co[vo])
    n = No[vo]
    assert float(d[n >= 10].max()) <= CTOL
    assert float((d * n).max()) <= 1e-3
    _say("gamma 0", seed, "max|dC| =", float(d.max()), "max|dS| =", float((d * n).max()))


@pytest.mark.parametrize("gamma", [0.3, 0.1, 0.6])
def test_decimal_gamma_threshold_matches_oracle(gamma):
    """Sec. 3.2's rule N >= gamma * m for a decimal gamma.  A's eroded mask is a 5 x 4 x 2 box
    (m = 40 against a larger B), so gamma * m is an integer and displacements with exactly
    N = gamma * m exist (box overlaps 1 x 4 x 1, 3 x 4 x 1, 3 x 4 x 2); they must be valid on both sides.
    Then a rotated random pair at the same gamma."""
    rng = np.random.default_rng(int(gamma * 100))
    A = rng.random((4, 6, 7)).astype(np.float32)          # (nz, ny, nx): eroded box 2 x 4 x 5
    B = rng.random((12, 12, 12)).astype(np.float32)
    _say("decimal gamma", gamma)
    with bd.Context(A, bd.dims_of(B), gamma=gamma) as ctx:
        Cg, Ng = ctx.evaluate_map(B, np.eye(3))
    Co, No, vo = _oracle_maps(A, B, np.eye(3), gamma=gamma)
    _compare_maps(Cg, Ng, Co, No, f"gamma{gamma}-box")
    edge = No == int(round(gamma * 40))
    assert edge.any() and vo[edge].all() and np.isfinite(Cg[edge]).all()
    assert not np.isfinite(Cg[No == int(round(gamma * 40)) - 1]).any()
    from scipy.ndimage import gaussian_filter
    sa = tuple(int(v) for v in rng.integers(6, 20, size=3))
    sb = tuple(int(v) for v in rng.integers(6, 20, size=3))
    A2 = gaussian_filter(rng.random(sa), 1.0).astype(np.float32)
    B2 = gaussian_filter(rng.random(sb), 1.0).astype(np.float32)
    R = _rand_rot(rng, 50)
    with bd.Context(A2, bd.dims_of(B2), gamma=gamma) as ctx:
        Cg, Ng = ctx.evaluate_map(B2, R)
    Co, No, _ = _oracle_maps(A2, B2, R, gamma=gamma)
    _compare_maps(Cg, Ng, Co, No, f"gamma{gamma}-rotated")


def test_repeated_rotation_reports_the_first_index():
    """Across rotations an exact tie goes to the smaller index: the same matrix given twice (in
    different slots of one launch and in a later launch) scores bit-identically, and the first
    copy is the reported best, as in the oracle."""
    pair = synth.config0()
    R = np.eye(3)
    rots = np.stack([_rand_rot(np.random.default_rng(5), 40), R, R, _rand_rot(np.random.default_rng(6), 40), R])
    with bd.Context(pair.A, pair.dims_b, batch=3) as ctx:
        per, best = ctx.evaluate(pair.B, rots)
    assert per[1].score == per[2].score == per[4].score
    assert tuple(per[1].shift) == tuple(per[2].shift) == tuple(per[4].shift)
    res, ob = O.evaluate(pair.A, pair.B, rots, P_xyz=pair.pad)
    assert ob == 1 and best.rot_index == 1


def test_kept_row_counts_match_overlap_bounds():
    """The minimum-overlap pruning (Sec. 3.2) keeps a displacement row (z, y) when the count of
    the moving mask over A's box rows shifted by (chi_z, chi_y) and all x reaches the threshold
    (an upper bound of N on that row), and a z-row likewise over all y and x.  The counters the
    benchmark reads must equal those rules recomputed from the oracle's mask, and every row
    that holds a valid displacement must be kept."""
    import math as _m
    pair = synth.config0()
    rng = np.random.default_rng(21)
    rots = np.stack([np.eye(3), _rand_rot(rng, 40), _rand_rot(rng, 70)])
    nza, nya, nxa = pair.A.shape
    nzb, nyb, nxb = pair.B.shape
    Wz, Wy = nza + nzb - 1, nya + nyb - 1
    want_z = want_r = 0
    maps = []
    with bd.Context(pair.A, pair.dims_b, pad=pair.pad, batch=2) as ctx:
        ctx.profile_reset()
        ctx.profile_enable(True)
        ctx.evaluate(pair.B, rots)
        kz, kr, nrot = ctx.profile_rows()
        ctx.profile_enable(False)
        for R in rots:
            maps.append(ctx.evaluate_map(pair.B, R)[0])
    assert nrot == len(rots)
    count_a = (nxa - 2) * (nya - 2) * (nza - 2)
    for R, Cg in zip(rots, maps):
        mb = O.moving_fields(pair.B, O.quantize_rotation(R)).mask
        thr = max(1, _m.ceil(0.5 * min(count_a, int(mb.sum()))))
        plane = mb.sum(axis=2)                       # [z][y] counts over x
        for zc in range(Wz):
            cz = zc - (nza - 1)
            lz, hz = max(1 + cz, 0), min(nza - 2 + cz, nzb - 1)
            zsum = int(plane[lz:hz + 1].sum()) if lz <= hz else 0
            want_z += zsum >= thr
            for yc in range(Wy):
                cy = yc - (nya - 1)
                ly, hy = max(1 + cy, 0), min(nya - 2 + cy, nyb - 1)
                rsum = int(plane[lz:hz + 1, ly:hy + 1].sum()) if (lz <= hz and ly <= hy) else 0
                kept = rsum >= thr
                want_r += kept
                if not kept:
                    assert not np.isfinite(Cg[zc, yc]).any(), (zc, yc)
    _say("kept rows", kz, kr, "expected", want_z, want_r)
    assert (kz, kr) == (want_z, want_r)


@pytest.mark.parametrize("seed", [107, 115, 119])
def test_fp64_correlation_meets_the_bar_at_every_overlap(seed):
    """With CSNGF_FP64 the transforms, the frequency-domain sum and the inverse run in double
    precision, so the small-overlap displacements that gamma = 0 admits (N down to 1) meet
    |dC| <= 1e-4 like all others: the pairs of test_gamma_zero_small_overlaps, every valid chi."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    sa = tuple(int(v) for v in rng.integers(3, 30, size=3))
    sb = tuple(int(v) for v in rng.integers(3, 30, size=3))
    A = gaussian_filter(rng.random(sa), 1.0).astype(np.float32)
    B = gaussian_filter(rng.random(sb), 1.0).astype(np.float32)
    R = _rand_rot(rng, 60)
    _say("fp64 gamma 0", seed, sa, sb)
    with bd.Context(A, bd.dims_of(B), gamma=0.0, fp64=True) as ctx:
        P = tuple(ctx.info().pad)
        Cg, Ng = ctx.evaluate_map(B, R)
    Co, No, _ = _oracle_maps(A, B, R, None, 0.0, P)
    _compare_maps(Cg, Ng, Co, No, f"fp64-gamma0-{seed}")
    n = No[np.isfinite(Co)]
    assert n.min() <= 3   # the case really holds tiny overlaps


@pytest.mark.parametrize("case", range(4))
def test_fp64_correlation_full_maps(case):
    """CSNGF_FP64 against the oracle: whole maps for random uneven pairs, both measures, a user
    mask on A, a mask on B, and the 32^3 pair with its known shift."""
    rng = np.random.default_rng(400 + case)
    from scipy.ndimage import gaussian_filter
    if case == 3:
        pair = synth.config0()
        A, B, R, P, mask_a, mask_b, measure = pair.A, pair.B, np.eye(3), pair.pad, None, None, "squared"
    else:
        sa = tuple(int(v) for v in rng.integers(5, 23, size=3))
        sb = tuple(int(v) for v in rng.integers(5, 23, size=3))
        A = gaussian_filter(rng.random(sa), 1.0).astype(np.float32)
        B = gaussian_filter(rng.random(sb), 1.0).astype(np.float32)
        R, P = _rand_rot(rng, 50), (0, 0, 0)
        mask_a = _mask_of_a(rng, sa, "ellipsoid-holes") if case == 1 else None
        mask_b = (rng.random(sb) > 0.03).astype(np.uint8) if case == 2 else None
        measure = "unsquared" if case == 2 else "squared"
    gamma = 0.25 if case == 2 else 0.5
    _say("fp64 map", case, A.shape, B.shape, measure, gamma)
    with bd.Context(A, bd.dims_of(B), pad=P, mask_a=mask_a, measure=measure, gamma=gamma, fp64=True) as ctx:
        Pused = tuple(ctx.info().pad)
        Cg, Ng = ctx.evaluate_map(B, R, mask_b=mask_b)
        per, best = ctx.evaluate(B, np.stack([R, np.eye(3)]), mask_b=mask_b)
    Co, No, _ = _oracle_maps(A, B, R, None if mask_b is None else mask_b.astype(bool), gamma, Pused,
                             mask_a=None if mask_a is None else mask_a.astype(bool), measure=measure)
    _compare_maps(Cg, Ng, Co, No, f"fp64-{case}")
    if case == 3:
        assert tuple(per[0].shift) == pair.true_shift


def test_padding_invariance_and_minimum_extent():
    rng = np.random.default_rng(9)
    A = rng.random((3, 4, 5)).astype(np.float32)
    B = rng.random((4, 3, 3)).astype(np.float32)
    _say("minimum extents")
    with bd.Context(A, bd.dims_of(B), gamma=0.0) as c1, bd.Context(A, bd.dims_of(B), gamma=0.0, pad=(16, 12, 16)) as c2:
        C1, N1 = c1.evaluate_map(B, np.eye(3))
        C2, N2 = c2.evaluate_map(B, np.eye(3))
    Co, No, _ = _oracle_maps(A, B, np.eye(3), gamma=0.0)
    _compare_maps(C1, N1, Co, No, "min-extent")
    assert np.array_equal(N1, N2)
    v = np.isfinite(C1)
    assert np.max(np.abs(C1[v] - C2[v])) <= CTOL


def test_config1_rotations_against_oracle():
    """The 96x96x64 pair with all 129 rotations (128 random and the generating one): the true
    rotation's whole map element by element, and every rotation's result against the oracle."""
    from parity_util import check_against_oracle_parallel
    pair = synth.config1()
    rots = pair.rotations
    _say("config1 evaluate", len(rots))
    with bd.Context(pair.A, pair.dims_b, pad=pair.pad) as ctx:
        per, best = ctx.evaluate(pair.B, rots)
        Cg, Ng = ctx.evaluate_map(pair.B, rots[pair.true_index])
    assert best.rot_index == pair.true_index
    assert tuple(best.shift) == pair.true_shift
    Co, No, _ = _oracle_maps(pair.A, pair.B, rots[pair.true_index], P=pair.pad)
    _compare_maps(Cg, Ng, Co, No, "config1-true")
    check_against_oracle_parallel(pair.A, pair.B, rots, per, best, P=pair.pad)
    _say("config1: all", len(rots), "rotations match the oracle")


def test_sign_invariance_and_repeatability_bit_identical():
    pair = synth.config0()
    rng = np.random.default_rng(3)
    R = _rand_rot(rng)
    with bd.Context(pair.A, pair.dims_b) as ctx:
        C1, N1 = ctx.evaluate_map(pair.B, R)
        C2, N2 = ctx.evaluate_map(-pair.B, R)
        C3, N3 = ctx.evaluate_map(pair.B, R)
    assert np.array_equal(C1, C2) and np.array_equal(N1, N2)
    assert np.array_equal(C1, C3) and np.array_equal(N1, N3)


def test_batch_invariance_bit_identical():
    pair = synth.config1(n_random=20)
    with bd.Context(pair.A, pair.dims_b, batch=1) as c1, bd.Context(pair.A, pair.dims_b, batch=7) as c7:
        p1, b1 = c1.evaluate(pair.B, pair.rotations)
        p7, b7 = c7.evaluate(pair.B, pair.rotations)
    for a, b in zip(p1, p7):
        assert a.score == b.score and tuple(a.shift) == tuple(b.shift) and a.overlap == b.overlap
    assert b1.rot_index == b7.rot_index == pair.true_index


@pytest.mark.parametrize("shape", [dict(slices=1), dict(slices=3), dict(slices=64), dict(final_groups=1),
                                   dict(final_groups=7), dict(final_groups=65535), dict(slices=5, final_groups=300)])
def test_launch_shapes_bit_identical(shape):
    # the launch shapes only split the same work: z slices per field-stage workgroup re-sample
    # the halo planes with the same arithmetic, and final-pass workgroups walk the same list
    pair = synth.config1(n_random=12)
    rng = np.random.default_rng(31)
    mask_a = (rng.random(pair.A.shape) < 0.9).astype(np.uint8)
    for ma in (None, mask_a):
        with bd.Context(pair.A, pair.dims_b, mask_a=ma) as c0, \
                bd.Context(pair.A, pair.dims_b, mask_a=ma, **shape) as c1:
            p0, b0 = c0.evaluate(pair.B, pair.rotations)
            p1, b1 = c1.evaluate(pair.B, pair.rotations)
            C0, N0 = c0.evaluate_map(pair.B, pair.rotations[3])
            C1, N1 = c1.evaluate_map(pair.B, pair.rotations[3])
        for a, b in zip(p0, p1):
            assert a.valid == b.valid and a.score == b.score and tuple(a.shift) == tuple(b.shift)
            assert a.overlap == b.overlap
        assert b0.rot_index == b1.rot_index and tuple(b0.shift) == tuple(b1.shift)
        assert np.array_equal(C0, C1) and np.array_equal(N0, N1)
    assert b0.rot_index >= 0


def test_edge_cases():
    rng = np.random.default_rng(4)
    A = rng.random((6, 6, 6)).astype(np.float32)
    B = rng.random((6, 6, 6)).astype(np.float32)
    with bd.Context(A, bd.dims_of(B)) as ctx:
        per, best = ctx.evaluate(B, np.zeros((0, 3, 3)))
        assert best.rot_index == -1
        bad = B.copy()
        bad[1, 2, 3] = np.inf
        with pytest.raises(bd.CsngfError) as ei:
            ctx.evaluate(bad, np.eye(3)[None])
        assert ei.value.code == bd.E_INVALID_ARG
        with pytest.raises(bd.CsngfError):
            ctx.evaluate(B, np.full((1, 3, 3), np.nan))
        # an empty mask on B leaves no valid displacement
        per, best = ctx.evaluate(B, np.eye(3)[None], mask_b=np.zeros(B.shape, np.uint8))
        assert best.rot_index == -1 and per[0].valid == 0 and math.isinf(best.score)
        with pytest.raises(bd.CsngfError) as ei:
            ctx.evaluate(B, np.eye(3)[None], mask_b=np.zeros(B.shape, np.uint8), allow_no_valid=False)
        assert ei.value.code == bd.E_NO_VALID_SHIFT
    # gamma = 1 with a rotation keeps only displacements covering the whole smaller mask
    with bd.Context(A, bd.dims_of(B), gamma=1.0) as ctx:
        R = _rand_rot(rng, 30)
        Cg, Ng = ctx.evaluate_map(B, R)
    Co, No, _ = _oracle_maps(A, B, R, gamma=1.0)
    _compare_maps(Cg, Ng, Co, No, "gamma1")


def test_device_pointer_path_with_torch_stream():
    import torch
    pair = synth.config0()
    dev = torch.device("cuda:0")
    A = torch.from_numpy(pair.A).to(dev)
    B = torch.from_numpy(pair.B).to(dev)
    s = torch.cuda.Stream()
    with bd.Context(A, pair.dims_b, stream=s) as ctx:
        per, best = ctx.evaluate(B, pair.rotations)
        W = tuple(ctx.info().map_dims)
        Cm = torch.empty((W[2], W[1], W[0]), dtype=torch.float32, device=dev)
        Nm = torch.empty((W[2], W[1], W[0]), dtype=torch.int64, device=dev)
        ctx.evaluate_map(B, np.eye(3), out=(Cm, Nm))
        s.synchronize()
        Ca, Na = ctx.evaluate_map(B, np.eye(3))   # outputs allocated by the binding
        assert Ca.device == dev and Na.dtype == torch.int64
        assert torch.equal(Ca, Cm) and torch.equal(Na, Nm)
        bad = B.clone()
        bad[0, 0, 0] = float("nan")
        with pytest.raises(bd.CsngfError):
            ctx.evaluate(bad, pair.rotations)
    with bd.Context(pair.A, pair.dims_b) as hctx:
        Ch, Nh = hctx.evaluate_map(pair.B, np.eye(3))
    assert np.array_equal(Cm.cpu().numpy(), Ch) and np.array_equal(Nm.cpu().numpy(), Nh)
    assert tuple(best.shift) == pair.true_shift


# ----------------------------------------------------------------------------- USNGF (Eq. (3))
def test_unsquared_field_stage_against_oracle():
    rng = np.random.default_rng(40)
    pair = synth.config0()
    R = _rand_rot(rng, 40)
    prod, m = bd.debug_fields(pair.B, R=R, unsquared=True)
    Rq = O.quantize_rotation(R)
    f = O.moving_fields(pair.B, Rq)
    Bh, _ = O.rotate_resample(pair.B, Rq)
    g = O.gradient(Bh)
    bound = _field_bound(pair.B, np.sum(g * g, axis=0), 1e-5)
    assert np.array_equal(m.astype(bool), f.mask)
    for k in range(3):
        assert np.all(np.abs(prod[k] - np.where(f.mask, f.n[k], 0.0)) <= bound)


@pytest.mark.parametrize("case", range(3))
def test_unsquared_maps_against_oracle(case):
    rng = np.random.default_rng(60 + case)
    if case == 0:
        pair = synth.config0()
        A, B, R, P = pair.A, pair.B, np.eye(3), pair.pad
    else:
        from scipy.ndimage import gaussian_filter
        sa = tuple(int(v) for v in rng.integers(6, 20, size=3))
        sb = tuple(int(v) for v in rng.integers(6, 20, size=3))
        A = gaussian_filter(rng.random(sa), 1.0).astype(np.float32)
        B = gaussian_filter(rng.random(sb), 1.0).astype(np.float32)
        R, P = _rand_rot(rng, 50), (0, 0, 0)
    _say("usngf", case, A.shape, B.shape)
    with bd.Context(A, bd.dims_of(B), pad=P, measure="unsquared") as ctx:
        Pused = tuple(ctx.info().pad)
        Cg, Ng = ctx.evaluate_map(B, R)
        Cn, Nn = ctx.evaluate_map(-B, R)
    fa = O.fixed_fields(A)
    fb = O.moving_fields(B, O.quantize_rotation(R))
    S, N = O.correlation_maps_fft(fa, fb, Pused, measure="unsquared")
    Co, _ = O.normalise(S, N, int(fa.mask.sum()), int(fb.mask.sum()))
    _compare_maps(Cg, Ng, Co, N, f"usngf{case}")
    # sign sensitivity of the unsquared measure: exact negation on the GPU as well
    v = np.isfinite(Cg)
    assert np.array_equal(np.isfinite(Cn), v) and np.array_equal(Cn[v], -Cg[v])
