"""Seeded synthetic inputs: determinism, shapes, dtypes and rotation validity."""
import numpy as np

from paper_2110_10156_amd import synth


def test_config0_deterministic_and_shaped():
    a, b = synth.config0(), synth.config0()
    assert a.A.shape == (32, 32, 32) and a.A.dtype == np.float32 and a.B.dtype == np.float32
    assert np.array_equal(a.A, b.A) and np.array_equal(a.B, b.B) and a.true_shift == b.true_shift
    assert all(-6 <= v <= 6 for v in a.true_shift)
    assert a.rotations.shape == (1, 3, 3) and np.array_equal(a.rotations[0], np.eye(3))
    assert float(a.A.max()) <= 1.0 + 1e-6


def test_rotations_are_proper():
    R = synth.random_rotations(64, 5)
    eye = np.einsum("nij,nkj->nik", R, R)
    assert np.allclose(eye, np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0)
    assert np.array_equal(R, synth.random_rotations(64, 5))


def test_euler_and_axis_angle_conventions():
    Rz = synth.axis_angle_matrix([0, 0, 1], np.pi / 2)
    assert np.allclose(Rz @ [1, 0, 0], [0, 1, 0])
    E = synth.euler_xyz_matrix(30, 20, 10)
    expect = (synth.axis_angle_matrix([1, 0, 0], np.radians(30))
              @ synth.axis_angle_matrix([0, 1, 0], np.radians(20))
              @ synth.axis_angle_matrix([0, 0, 1], np.radians(10)))
    assert np.allclose(E, expect)


def test_intensity_map_is_non_monotonic():
    v = np.linspace(0, 1, 101)
    d = np.diff(synth.intensity_map_f(v))
    assert (d > 0).any() and (d < 0).any()


def test_config1_truth_appended():
    p = synth.config1(n_random=4)
    assert p.A.shape == (64, 96, 96) and p.rotations.shape == (5, 3, 3)
    assert p.true_index == 4 and np.array_equal(p.rotations[4], p.true_rotation)
    assert all(-15 <= v <= 15 for v in p.true_shift)


def test_euler_matrices_vectorised_equals_single():
    rng = np.random.default_rng(9)
    ang = rng.uniform(-200.0, 200.0, size=(50, 3))
    many = synth.euler_xyz_matrices(ang)
    one = np.stack([synth.euler_xyz_matrix(*a) for a in ang])
    assert many.shape == (50, 3, 3)
    assert np.max(np.abs(many - one)) < 1e-14
    assert np.allclose(many @ np.transpose(many, (0, 2, 1)), np.eye(3), atol=1e-14)
