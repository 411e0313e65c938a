"""Pins of the oracle's Pipe-Menon density compensation (CPU)."""

import math

import numpy as np

from oracle import dcf, gridding


def _i0_series(x):
    """I0 by its power series sum (x^2/4)^m / (m!)^2, written out."""
    t, s, m = 1.0, 1.0, 0
    while t > 1e-18 * s:
        m += 1
        t *= (x * x / 4.0) / (m * m)
        s += t
    return s


def test_points_on_a_shifted_full_grid_give_the_closed_form_constant():
    # one point half a cell past every node of a 16^3 fine grid (offsets
    # then stay clear of the support edge): a point's nodes sit at offsets
    # u = +-0.5, +-1.5, +-2.5, so spreading 1 gives S^3 on every node and
    # interpolating it back gives S^6, S = sum_u phi~(u)
    g = gridding.Grid((8, 8, 8))
    nf = g.nf[0]
    m = np.arange(nf) + 0.5
    kz, ky, kx = np.meshgrid(m, m, m, indexing="ij")
    k = 2 * np.pi * np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1) / nf
    S = sum(_i0_series(g.beta * math.sqrt(1.0 - (2.0 * u / g.W) ** 2))
            for u in (-2.5, -1.5, -0.5, 0.5, 1.5, 2.5))
    S /= _i0_series(g.beta)
    w1 = dcf.pipe_menon(g, k, 1)
    assert np.allclose(w1, 1.0 / S ** 6, rtol=1e-12, atol=0)
    assert np.allclose(dcf.pipe_menon(g, k, 4), 1.0 / S ** 6, rtol=1e-12, atol=0)


def test_duplicated_points_halve_the_weights():
    g = gridding.Grid((10, 12, 9))
    k = np.random.default_rng(3).uniform(-np.pi, np.pi, (700, 3))
    for it in (1, 3):
        w = dcf.pipe_menon(g, k, it)
        w2 = dcf.pipe_menon(g, np.concatenate([k, k]), it)
        assert np.allclose(w2[:700], w / 2, rtol=1e-12)
        assert np.allclose(w2[700:], w / 2, rtol=1e-12)


def test_shift_by_whole_fine_cells_is_invariant():
    g = gridding.Grid((10, 12, 9))
    k = np.random.default_rng(4).uniform(-np.pi, np.pi, (500, 3))
    step = 2 * np.pi / np.array(g.nf[::-1], dtype=np.float64)   # one cell per axis (x, y, z)
    w = dcf.pipe_menon(g, k, 3)
    assert np.allclose(dcf.pipe_menon(g, k + step * np.array([3, -2, 5]), 3), w, rtol=1e-11)


def test_iteration_drives_the_convolved_weights_towards_one():
    g = gridding.Grid((16, 16, 16))
    import workloads as wl
    k, _ = wl.spiral_trajectory(6, 8, 300)
    k = k.astype(np.float64)
    r = []
    for it in (1, 4, 12):
        w = dcf.pipe_menon(g, k, it)
        r.append(np.sqrt(np.mean((dcf.convolve(g, k, w) - 1.0) ** 2)))
    assert r[1] < r[0] and r[2] < r[1]
    assert r[2] < 0.1
