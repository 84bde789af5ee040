"""Host-side pieces of bench.py: the byte and flop models the roofline objects divide by."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plan_factorisation_matches_the_engine():
    # odd radices first, then 8, 4, 2 (the compile-time plans of the FFT engine)
    assert bench.plan_radices(220) == [11, 5, 4]
    assert bench.plan_radices(352) == [11, 8, 4]
    assert bench.plan_radices(512) == [8, 8, 8]
    assert bench.plan_radices(96) == [3, 8, 4]


def test_flop_model_hand_counts():
    # radix-11 butterfly: pairs (4h), y0 (2h), 2h^2 fma per A_k and B_k, outputs (4h), h = 5
    assert bench.dft_flops(11, False) == 250 and bench.dft_flops(11, True) == 230
    assert bench.dft_flops(5, False) == 52 and bench.dft_flops(4, False) == 16 and bench.dft_flops(8, False) == 56
    # 220 = 11 * 5 * 4: 20 radix-11 (no twiddles), 44 radix-5 and 55 radix-4 with 4 and 3 twiddles
    assert bench.transform_flops(220, True) == 20 * 230 + 44 * (52 + 24) + 55 * (16 + 18)
    assert bench.transform_flops(220, False) == 20 * 250 + 44 * (52 + 24) + 55 * (16 + 18)
    # the z pass of the 176x176x110 pair at 352x352x220: 352 * 176 pencils, 6 forward + MAC + 1 inverse
    per_col = 6 * (9814 + 8 * 220) + 10214
    assert bench.zpass_flops((176, 176, 110), (352, 352, 220)) == 352 * 176 * per_col


def test_byte_model_kept_rows():
    kb = bench.kernel_bytes((176, 176, 110), (176, 176, 110), (352, 352, 220), 16.0, (109.0, 13007.7))
    x2 = 6 * 108 * 352 * 176 * 8
    assert kb["y_forward"] == 6 * 108 * 174 * 176 * 8 + x2
    assert abs(kb["z_mac_inverse"] - (x2 + 6 * 220 * 352 * 176 * 8 / 16 + 109 * 352 * 176 * 8)) < 1


def test_byte_model_mask_runs():
    # without user masks the moving masks are runs of x per row (8 B), and the field stage
    # writes no mask; with a mask the field stage writes one byte per voxel and the table reads it
    dims, P = (176, 176, 110), (352, 352, 220)
    vox, x1 = 176 * 176 * 110, 6 * 108 * 174 * 176 * 8
    r = bench.kernel_bytes(dims, dims, P, 16.0)
    m = bench.kernel_bytes(dims, dims, P, 16.0, runs=False)
    assert r["fields_x"] == 4 * vox + x1 and m["fields_x"] == 5 * vox + x1
    assert m["overlap_sat"] - r["overlap_sat"] == vox - 2 * 8 * 176 * 110


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
