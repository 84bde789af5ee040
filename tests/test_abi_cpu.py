"""The C-ABI library: it loads, exports every symbol the headers declare, and rejects bad
arguments (no GPU needed for any of this)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2110_10156_amd import binding as bd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def _declared_functions():
    names = set()
    for h in ("csngf.h", "csngf_debug.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(csngf_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = bd.lib()
    declared = _declared_functions()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(L, name), name
        assert name in bd.SIGNATURES, name


def test_struct_sizes_match_header_layout():
    assert C.sizeof(bd.Params) == 48
    assert bd.Params.gamma.offset == 8 and bd.Params.pad.offset == 16 and bd.Params.flags.offset == 32
    assert bd.Params.slices.offset == 36 and bd.Params.final_groups.offset == 40 and bd.Params.reserved.offset == 44
    assert C.sizeof(bd.RotResult) == 32
    assert C.sizeof(bd.Best) == 32 + 72
    assert C.sizeof(bd.Dims) == 12


def test_default_params():
    p = bd.default_params()
    assert p.struct_size == C.sizeof(bd.Params)
    assert abs(p.eps - 1e-5) < 1e-12 and p.gamma == 0.5
    assert list(p.pad) == [0, 0, 0] and p.batch == 0 and p.flags == 0
    assert p.slices == 0 and p.final_groups == 0 and p.reserved == 0


@pytest.mark.parametrize("L,ok", [(8, 1), (64, 1), (220, 1), (352, 1), (192, 1), (110, 1), (440, 1), (512, 1),
                                  (6, 0), (13, 0), (26, 0), (514, 0), (1024, 0), (63, 0), (0, 0), (-4, 0)])
def test_supported_lengths(L, ok):
    assert bd.lib().csngf_supported_length(L) == ok


def _create(A, dB, mask=None, params=None):
    h = C.c_void_p()
    rc = bd.lib().csngf_create(None if A is None else A.ctypes.data, bd.dims_of(A) if A is not None else bd.Dims(8, 8, 8),
                               None if mask is None else mask.ctypes.data, dB,
                               None if params is None else C.byref(params), C.byref(h))
    return rc, h


def test_create_rejects_bad_arguments_before_touching_a_device():
    A = np.zeros((8, 8, 8), dtype=np.float32)
    dB = bd.Dims(8, 8, 8)
    assert _create(None, dB)[0] == bd.E_INVALID_ARG
    assert b"NULL" in bd.lib().csngf_last_error()
    assert _create(np.zeros((2, 8, 8), np.float32), dB)[0] == bd.E_INVALID_ARG
    assert _create(A, bd.Dims(8, 2, 8))[0] == bd.E_INVALID_ARG
    bad = A.copy()
    bad[3, 3, 3] = np.nan
    assert _create(bad, dB)[0] == bd.E_INVALID_ARG
    assert b"non-finite" in bd.lib().csngf_last_error()
    p = bd.default_params()
    p.gamma = 1.5
    assert _create(A, dB, params=p)[0] == bd.E_INVALID_ARG
    p = bd.default_params()
    p.eps = 0.0
    assert _create(A, dB, params=p)[0] == bd.E_INVALID_ARG
    p = bd.default_params()
    p.struct_size = 4
    assert _create(A, dB, params=p)[0] == bd.E_INVALID_ARG
    for batch in (-1, 256):   # slots are packed in 8 bits in the final pass's work list
        p = bd.default_params()
        p.batch = batch
        assert _create(A, dB, params=p)[0] == bd.E_INVALID_ARG
    for field, bad in (("slices", -1), ("slices", 65), ("final_groups", -1), ("final_groups", 65536),
                       ("reserved", 1)):
        p = bd.default_params()
        setattr(p, field, bad)
        assert _create(A, dB, params=p)[0] == bd.E_INVALID_ARG, field
        assert field.encode() in bd.lib().csngf_last_error()
    p = bd.default_params()
    p.pad[0] = 10  # < 8 + 8 - 1
    assert _create(A, dB, params=p)[0] == bd.E_INVALID_ARG
    p = bd.default_params()
    p.pad[0] = 26  # 2 * 13: not built
    assert _create(A, dB, params=p)[0] == bd.E_UNSUPPORTED
    assert _create(np.zeros((8, 8, 600), np.float32), dB)[0] == bd.E_UNSUPPORTED


def test_other_entry_points_reject_null():
    L = bd.lib()
    assert L.csngf_destroy(None) == bd.E_INVALID_ARG
    assert L.csngf_evaluate(None, None, None, None, 0, None, None) == bd.E_INVALID_ARG
    assert L.csngf_evaluate_map(None, None, None, None, None, None) == bd.E_INVALID_ARG
    assert L.csngf_set_stream(None, None) == bd.E_INVALID_ARG
    assert L.csngf_get_info(None, None) == bd.E_INVALID_ARG
    assert L.csngf_profile_enable(None, 1) == bd.E_INVALID_ARG
    assert L.csngf_default_params(None) == bd.E_INVALID_ARG
    assert L.csngf_debug_fft(None, None, 64, 1, 0, None) == bd.E_INVALID_ARG
    x = C.c_void_p(16)
    assert L.csngf_debug_fft(x, x, 26, 1, 0, None) == bd.E_UNSUPPORTED


@pytest.mark.skipif(_gpu_present(), reason="a GPU is visible")
def test_no_device_is_reported():
    A = np.random.default_rng(0).random((8, 8, 8)).astype(np.float32)
    rc, h = _create(A, bd.Dims(8, 8, 8))
    assert rc == bd.E_NO_DEVICE
    # a user mask on A passes argument checking (it is supported) and then needs a device
    assert _create(A, bd.Dims(8, 8, 8), mask=np.ones(A.shape, np.uint8))[0] == bd.E_NO_DEVICE
    assert b"device" in bd.lib().csngf_last_error()
    with pytest.raises(bd.CsngfError) as ei:
        bd.Context(A, (8, 8, 8))
    assert ei.value.code == bd.E_NO_DEVICE


def test_automatic_fft_size_prefers_fixed_length_plans():
    """pad = 0: the smallest supported length >= n_A + n_B - 1, or the smallest one with a
    compile-time plan when that is at most 1.5x as long (csngf_footprint reports the choice)."""
    cases = {(32, 32, 32): 64,       # 63 -> 64 (planned)
             (100, 100, 100): 220,   # 199 -> 200 has no fixed plan; 220 does
             (129, 129, 129): 352,   # 257 -> 264 unplanned; 352 <= 1.5 * 264
             (201, 201, 201): 440,   # 401 -> 420 unplanned; 440
             (96, 96, 64): 192}      # x, y: 191 -> 192; z below
    for dims, want in cases.items():
        P = bd.footprint(dims, dims)[2]
        assert P[0] == want, (dims, P)
    assert bd.footprint((96, 96, 64), (96, 96, 64))[2][2] == 128
    assert bd.footprint((176, 176, 110), (176, 176, 110))[2] == (352, 352, 220)
    # an explicit pad is kept as given
    assert bd.footprint((100, 100, 100), (100, 100, 100), pad=(200, 200, 200))[2] == (200, 200, 200)


def test_footprint_per_context_and_per_slot_bytes():
    """The per-context figure is A's six conjugate spectra ([6][Pz][Py][Hp] complex64) plus B's
    brick copy (5^3 floats per brick of 4^3 cells, ceil((n - 1) / 4) bricks per axis); the
    per-slot figure grows with the rotation workspaces and is the same for FP32 and FP64 apart
    from the transform buffers."""
    spec, slot, P = bd.footprint((176, 176, 110), (176, 176, 110))
    assert P == (352, 352, 220)
    bricks = 44 * 44 * 28
    assert spec == 6 * 220 * 352 * 176 * 8 + 4 * 125 * bricks
    # X1/Y3 and X2/Y4 buffers dominate a slot: at least (6 * 108 * 352 + 6 * 108 * 174) * 176 bins
    assert slot >= 8 * 6 * 108 * (352 + 174) * 176
    # a 3-voxel axis still gets one brick; rows hold Px/2 bins padded to the 16-bin tile
    spec3, _, P3 = bd.footprint((3, 3, 3), (3, 3, 3))
    hp = -(-(P3[0] // 2) // 16) * 16
    assert spec3 == 6 * P3[2] * P3[1] * hp * 8 + 4 * 125


def test_noalloc_pyramid_rejects_bad_and_oversized_arguments():
    """The allocation-free pyramid entry point validates before touching a device: NULL
    pointers, bad sigma or factor, and inputs whose intermediates exceed the fixed scratch."""
    L = bd.lib()
    od = bd.Dims()
    x = C.c_void_p(256)
    assert L.csngf_smooth_downsample_noalloc(None, bd.Dims(8, 8, 8), 1.0, 1, x, C.byref(od), None) == bd.E_INVALID_ARG
    assert L.csngf_smooth_downsample_noalloc(x, bd.Dims(8, 8, 8), -1.0, 1, x, C.byref(od), None) == bd.E_INVALID_ARG
    assert L.csngf_smooth_downsample_noalloc(x, bd.Dims(8, 8, 8), 1.0, 0, x, C.byref(od), None) == bd.E_INVALID_ARG
    # output dims can be queried without an output
    assert L.csngf_smooth_downsample_noalloc(x, bd.Dims(9, 8, 7), 1.0, 2, None, C.byref(od), None) == bd.OK
    assert (od.nx, od.ny, od.nz) == (5, 4, 4)
    # 256^3 at factor 1: 2 x 64 MiB of intermediates, above the 32 MiB scratch
    rc = L.csngf_smooth_downsample_noalloc(x, bd.Dims(256, 256, 256), 1.0, 1, x, C.byref(od), None)
    assert rc == bd.E_UNSUPPORTED and b"scratch" in L.csngf_last_error()
    # the largest cube that fits at factor 1: 2 n^3 floats <= 8 Mi (n = 161); 162 does not
    rc = L.csngf_smooth_downsample_noalloc(x, bd.Dims(162, 162, 162), 1.0, 1, x, C.byref(od), None)
    assert rc == bd.E_UNSUPPORTED
    if not _gpu_present():   # past the size check, the call needs a device
        for dims in (bd.Dims(161, 161, 161), bd.Dims(176, 176, 110)):
            assert L.csngf_smooth_downsample_noalloc(x, dims, 1.0, 1, x, C.byref(od), None) == bd.E_NO_DEVICE
