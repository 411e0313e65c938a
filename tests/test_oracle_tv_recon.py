"""Pins of the TV and initialiser oracles (CPU only).

TV: closed forms (flat image, linear ramp, one step edge), a pure-Python
loop over voxels on a tiny image, and central differences of the value for
the gradient.  Initialisers: conjugate gradients against a dense solve of
the normal equations built from the operator's definition, the
full-Cartesian case where the normal operator is N_vox times the identity
(CG exact in one step, the scaled adjoint returns the true image), and the
optimality of the adjoint's scale.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import mrf, nudft, recon, tv


def _cimg(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


# ------------------------------------------------------------------------ TV
def test_tv_flat_image():
    x = np.full((2, 3, 4, 5), 0.7 - 0.2j)
    eps = 0.3
    assert tv.value(x, eps) == pytest.approx(2 * 60 * eps, rel=1e-14)
    assert np.max(np.abs(tv.grad(x, eps))) == 0.0


def test_tv_linear_ramp_along_x():
    K, nz, ny, nx = 2, 3, 4, 6
    a, eps = 0.25, 0.1
    ramp = a * np.arange(nx) * (1 + 1j) / math.sqrt(2)     # |step| = a
    x = np.broadcast_to(ramp, (K, nz, ny, nx)).copy()
    expect = K * nz * ny * ((nx - 1) * math.sqrt(a * a + eps * eps) + eps)
    assert tv.value(x, eps) == pytest.approx(expect, rel=1e-13)


def test_tv_step_edge_along_z_without_smoothing():
    K, nz, ny, nx = 1, 6, 3, 4
    x = np.zeros((K, nz, ny, nx), dtype=complex)
    x[:, 3:] = 2.0j
    # only the plane z = 2 has a nonzero difference, of modulus 2
    assert tv.value(x, 0.0) == pytest.approx(2.0 * ny * nx, rel=1e-14)


def test_tv_matches_voxel_loop():
    x = _cimg((2, 3, 4, 5), 7)
    eps = 0.05
    K, nz, ny, nx = x.shape
    total = 0.0
    for k, z, y, xx in itertools.product(range(K), range(nz), range(ny), range(nx)):
        s = eps * eps
        if xx + 1 < nx:
            s += abs(x[k, z, y, xx + 1] - x[k, z, y, xx]) ** 2
        if y + 1 < ny:
            s += abs(x[k, z, y + 1, xx] - x[k, z, y, xx]) ** 2
        if z + 1 < nz:
            s += abs(x[k, z + 1, y, xx] - x[k, z, y, xx]) ** 2
        total += math.sqrt(s)
    assert tv.value(x, eps) == pytest.approx(total, rel=1e-13)


def test_tv_gradient_central_differences():
    x = _cimg((2, 4, 3, 5), 8)
    eps, h = 0.2, 1e-6
    g = tv.grad(x, eps)
    rng = np.random.default_rng(9)
    for _ in range(12):
        idx = tuple(int(rng.integers(0, n)) for n in x.shape)
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            xp = x.copy(); xp[idx] += unit * h
            xm = x.copy(); xm[idx] -= unit * h
            fd = (tv.value(xp, eps) - tv.value(xm, eps)) / (2 * h)
            assert fd == pytest.approx(part(g[idx]), abs=1e-7), (idx, unit)


# ----------------------------------------------------------------- recon
def _small_problem(seed, K=2, C=2, M=300, shape=(4, 4, 4), T=3):
    g = np.random.default_rng(seed)
    k = g.uniform(-np.pi, np.pi, (M, 3))
    frame = g.integers(0, T, M)
    smaps = _cimg((C,) + shape, seed + 1) / 3
    V = _cimg((T, K), seed + 2) / 2
    w = g.uniform(0.5, 1.5, M)
    y = _cimg((C, M), seed + 3)
    return k, frame, smaps, V, w, y


def _dense_operator(k, frame, smaps, V, shape):
    """A[(c, j), (kk, voxel)] = V[t_j, kk] S_c[voxel] exp(-i k_j . n) from the
    definition of the forward operator."""
    nz, ny, nx = shape
    mz, my, mx = np.meshgrid(nudft.modes(nz), nudft.modes(ny), nudft.modes(nx), indexing="ij")
    n = np.stack([mx.ravel(), my.ravel(), mz.ravel()], -1)          # (x, y, z) per voxel
    E = np.exp(-1j * (k @ n.T))                                      # [M, N]
    C, K = smaps.shape[0], V.shape[1]
    A = np.zeros((C * k.shape[0], K * n.shape[0]), dtype=complex)
    for c in range(C):
        for kk in range(K):
            A[c * k.shape[0]:(c + 1) * k.shape[0], kk * n.shape[0]:(kk + 1) * n.shape[0]] = \
                V[frame, kk][:, None] * E * smaps[c].ravel()[None, :]
    return A


@pytest.mark.parametrize("lam", [0.0, 5.0])
def test_cg_reaches_dense_solution(lam):
    shape, K = (4, 4, 4), 2
    k, frame, smaps, V, w, y = _small_problem(11)
    op = mrf.Nufft(shape, "direct")
    A = _dense_operator(k, frame, smaps, V, shape)
    Wd = np.tile(w, smaps.shape[0])
    Nmat = A.conj().T @ (Wd[:, None] * A) + lam * np.eye(A.shape[1])
    bvec = A.conj().T @ (Wd * y.ravel())
    xs = np.linalg.solve(Nmat, bvec).reshape((K,) + shape)
    # dimension K N_vox = 128: CG is exact after 128 steps in exact arithmetic
    x, hist = recon.cg(op, y, smaps, V, frame, k, np.zeros((K,) + shape), 128, w=w, lam=lam)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert hist[-1] <= 1e-16 * hist[0]
    # the normal operator and right-hand side themselves
    xt = _cimg((K,) + shape, 12)
    Nx = recon.normal(op, xt, smaps, V, frame, k, w, lam)
    assert np.linalg.norm(Nx.ravel() - Nmat @ xt.ravel()) <= 1e-11 * np.linalg.norm(Nx)
    b = recon.rhs(op, y, smaps, V, frame, k, K, w)
    assert np.linalg.norm(b.ravel() - bvec) <= 1e-11 * np.linalg.norm(bvec)


def _cartesian(shape):
    nz, ny, nx = shape
    mz, my, mx = np.meshgrid(nudft.modes(nz), nudft.modes(ny), nudft.modes(nx), indexing="ij")
    return np.stack([2 * np.pi * mx / nx, 2 * np.pi * my / ny, 2 * np.pi * mz / nz], -1).reshape(-1, 3)


def _unit_coils(shape, C, seed):
    s = _cimg((C,) + shape, seed)
    return s / np.sqrt(np.sum(np.abs(s) ** 2, axis=0, keepdims=True))


@pytest.mark.parametrize("lam", [0.0, 3.0])
def test_cg_full_cartesian_one_step(lam):
    shape = (4, 4, 4)
    nvox = 64
    k = _cartesian(shape)
    frame = np.zeros(k.shape[0], dtype=int)
    smaps = _unit_coils(shape, 3, 21)
    V = np.array([[1.0 + 0j]])
    op = mrf.Nufft(shape, "direct")
    xt = _cimg((1,) + shape, 22)
    y = mrf.forward(op, xt, smaps, [0, 1, 2], V, frame, k)
    x, hist = recon.cg(op, y, smaps, V, frame, k, np.zeros_like(xt), 1, lam=lam)
    assert np.max(np.abs(x - xt * nvox / (nvox + lam))) <= 1e-12 * np.max(np.abs(xt))
    assert hist[1] <= 1e-24 * hist[0]


def test_scaled_adjoint_full_cartesian_is_exact():
    shape = (4, 4, 4)
    k = _cartesian(shape)
    frame = np.zeros(k.shape[0], dtype=int)
    smaps = _unit_coils(shape, 2, 31)
    V = np.array([[1.0 + 0j]])
    op = mrf.Nufft(shape, "direct")
    xt = _cimg((1,) + shape, 32)
    y = mrf.forward(op, xt, smaps, [0, 1], V, frame, k)
    x0, s = recon.scaled_adjoint(op, y, smaps, V, frame, k, 1)
    assert s == pytest.approx(1.0 / 64, rel=1e-12)
    assert np.max(np.abs(x0 - xt)) <= 1e-12 * np.max(np.abs(xt))


def test_scaled_adjoint_scale_is_optimal():
    shape, K = (4, 4, 4), 2
    k, frame, smaps, V, w, y = _small_problem(41)
    op = mrf.Nufft(shape, "direct")
    x0, s = recon.scaled_adjoint(op, y, smaps, V, frame, k, K, w)
    z = x0 / s
    Az = mrf.forward(op, z, smaps, [0, 1], V, frame, k)

    def obj(t):
        return float(np.sum(w[None, :] * np.abs(y - t * Az) ** 2))
    assert obj(s) < obj(s * 1.001) and obj(s) < obj(s * 0.999)
    # the derivative in t vanishes at s
    assert abs(obj(s * (1 + 1e-5)) - obj(s * (1 - 1e-5))) <= 1e-8 * obj(s)
