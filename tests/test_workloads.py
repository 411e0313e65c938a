"""The seeded input generators: ranges, structure and determinism (CPU)."""

import numpy as np

import workloads as wl


def test_spiral_trajectory_shape_range_and_frames():
    traj, frame = wl.spiral_trajectory(3, 4, 100)
    assert traj.shape == (1200, 3) and traj.dtype == np.float32
    assert frame.dtype == np.int32 and np.all(np.diff(frame) >= 0)
    assert np.all(np.bincount(frame) == 400)
    assert np.all(traj >= -np.pi) and np.all(traj < np.pi)
    # every arm starts at the k-space centre (hot bins, as in MRF spirals)
    assert np.allclose(traj.reshape(12, 100, 3)[:, 0], 0.0)
    r = np.linalg.norm(traj.reshape(12, 100, 3), axis=2)
    assert np.allclose(r[:, -1], wl.KMAX, rtol=1e-6)


def test_generators_are_deterministic():
    a, _ = wl.spiral_trajectory(2, 2, 50)
    b, _ = wl.spiral_trajectory(2, 2, 50)
    assert np.array_equal(a, b)
    assert np.array_equal(wl.subspace_basis(30, 4, 7), wl.subspace_basis(30, 4, 7))
    assert np.array_equal(wl.phantom((8, 9, 10), 2, 3), wl.phantom((8, 9, 10), 2, 3))


def test_coil_maps_unit_rss():
    s = wl.coil_maps((10, 12, 14), 6, 1)
    assert s.shape == (6, 10, 12, 14) and s.dtype == np.complex64
    assert np.allclose(np.sqrt(np.sum(np.abs(s) ** 2, axis=0)), 1.0, atol=1e-5)


def test_subspace_basis_orthonormal():
    v = wl.subspace_basis(200, 5, 2).astype(np.complex128)
    assert np.allclose(v.conj().T @ v, np.eye(5), atol=1e-6)


def test_phantom_structure():
    x = wl.phantom((20, 22, 24), 3, 4)
    assert x.shape == (3, 20, 22, 24) and x.dtype == np.complex64
    assert abs(x[:, 0, 0, 0]).max() < 1e-3          # background is zero
    assert abs(x[:, 10, 11, 12]).max() > 0.1        # head is not


def test_coil_minibatch_is_a_permutation_per_epoch():
    got = np.concatenate([wl.coil_minibatch(32, 4, 3, s) for s in range(8)])
    assert sorted(got.tolist()) == list(range(32))
