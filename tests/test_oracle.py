"""Pins of the CPU FP64 oracle to things other than itself (CPU only).

Each test checks the oracle against a library routine on a special case, a
closed form, an invariant, quadrature or brute force, chosen so that a
dropped term, a wrong sign, a swapped axis or a transposed operand in the
oracle fails at least one of them.
"""

import os

import numpy as np
import pytest
import scipy.integrate

from oracle import gridding, kernel, mrf, nudft

HERE = os.path.dirname(os.path.abspath(__file__))


def _img(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _on_grid_points(shape):
    """All k = 2 pi m / N for m in the mode set, as [M, 3] (kx, ky, kz)."""
    nz, ny, nx = shape
    mz, my, mx = np.meshgrid(nudft.modes(nz), nudft.modes(ny), nudft.modes(nx),
                             indexing="ij")
    k = np.stack([2 * np.pi * mx / nx, 2 * np.pi * my / ny, 2 * np.pi * mz / nz], -1)
    return k.reshape(-1, 3)


# ---------------------------------------------------------------- direct NUDFT
@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 3, 7), (6, 6, 6)])
def test_type2_on_grid_is_centred_fft(shape):
    f = _img(shape, 1)
    c = nudft.type2(f, _on_grid_points(shape)).reshape(shape)
    ref = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(f)))
    assert np.max(np.abs(c - ref)) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 3, 7)])
def test_type1_on_grid_is_centred_ifft(shape):
    c = _img(shape, 2)
    f = nudft.type1(c.ravel(), _on_grid_points(shape), shape)
    ref = np.fft.fftshift(np.fft.ifftn(np.fft.ifftshift(c))) * np.prod(shape)
    assert np.max(np.abs(f - ref)) < 1e-11 * np.max(np.abs(ref))


def test_parseval_on_grid():
    shape = (6, 5, 4)
    f = _img(shape, 3)
    c = nudft.type2(f, _on_grid_points(shape))
    assert abs(np.sum(np.abs(c) ** 2) - np.prod(shape) * np.sum(np.abs(f) ** 2)) \
        < 1e-10 * np.sum(np.abs(c) ** 2)


def _load_golden(name):
    rows, meta = [], {}
    with open(os.path.join(HERE, "golden", name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] in ("shape", "index"):
                meta[tok[0]] = tuple(int(t) for t in tok[1:])
            else:
                rows.append([float(t) for t in tok])
    return meta, np.array(rows)


def test_delta_image_golden():
    meta, rows = _load_golden("delta_image_type2.txt")
    f = np.zeros(meta["shape"], dtype=np.complex128)
    f[meta["index"]] = 1.0
    k = rows[:, :3] * np.pi
    c = nudft.type2(f, k)
    assert np.max(np.abs(c - (rows[:, 3] + 1j * rows[:, 4]))) < 1e-12


def test_single_point_at_origin_type1_is_constant():
    f = nudft.type1(np.array([2.5 - 1j]), np.zeros((1, 3)), (3, 4, 5))
    assert np.allclose(f, 2.5 - 1j, atol=1e-14)


def test_direct_vs_pure_python_loops():
    shape = (3, 4, 5)
    f = _img(shape, 4)
    g = np.random.default_rng(5)
    k = g.uniform(-np.pi, np.pi, (7, 3))
    c = g.standard_normal(7) + 1j * g.standard_normal(7)
    nz, ny, nx = shape
    ref2 = np.zeros(7, dtype=np.complex128)
    ref1 = np.zeros(shape, dtype=np.complex128)
    for j in range(7):
        for iz in range(nz):
            for iy in range(ny):
                for ix in range(nx):
                    ph = (k[j, 0] * (ix - nx // 2) + k[j, 1] * (iy - ny // 2)
                          + k[j, 2] * (iz - nz // 2))
                    ref2[j] += f[iz, iy, ix] * complex(np.cos(ph), -np.sin(ph))
                    ref1[iz, iy, ix] += c[j] * complex(np.cos(ph), np.sin(ph))
    assert np.max(np.abs(nudft.type2(f, k) - ref2)) < 1e-12
    assert np.max(np.abs(nudft.type1(c, k, shape) - ref1)) < 1e-12


def test_direct_adjoint_identity():
    shape = (7, 6, 5)
    f = _img(shape, 6)
    g = np.random.default_rng(7)
    k = g.uniform(-np.pi, np.pi, (300, 3))
    c = g.standard_normal(300) + 1j * g.standard_normal(300)
    lhs = np.vdot(c, nudft.type2(f, k))
    rhs = np.vdot(nudft.type1(c, k, shape), f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_type1_subset_selection():
    shape = (6, 7, 8)
    g = np.random.default_rng(8)
    k = g.uniform(-np.pi, np.pi, (200, 3))
    c = g.standard_normal(200) + 1j * g.standard_normal(200)
    full = nudft.type1(c, k, shape)
    sel = ([1, 4], [0, 3, 6], [2, 7])
    part = nudft.type1(c, k, shape, sel=sel)
    assert np.allclose(part, full[np.ix_(*sel)], atol=1e-12)


# ---------------------------------------------------------------- the kernel
def test_i0_matches_power_series():
    x = np.linspace(0.0, 14.0, 57)
    series = np.zeros_like(x)
    term = np.ones_like(x)
    for m in range(80):
        series += term
        term = term * (x * x / 4.0) / ((m + 1) ** 2)
    u = 3.0 * np.sqrt(np.clip(1 - (x / 14.0) ** 2, 0, 1))  # any |u| <= W/2
    b = 14.0
    val = kernel.phi(u, 6, b)
    assert np.allclose(val, series, rtol=1e-13)


@pytest.mark.parametrize("W,sigma", [(6, 2.0), (4, 2.0), (8, 2.0), (6, 1.5)])
def test_phi_hat_matches_quadrature(W, sigma):
    b = kernel.beta(W, sigma)
    xi = np.linspace(-0.5 / sigma, 0.5 / sigma, 9)
    got = kernel.phi_hat(xi, W, b)
    for x0, gv in zip(xi, got):
        val, _ = scipy.integrate.quad(
            lambda u: kernel.phi(np.array([u]), W, b)[0] * np.cos(2 * np.pi * x0 * u),
            -W / 2, W / 2, limit=200, epsabs=0, epsrel=1e-13)
        assert abs(val - gv) < 1e-11 * abs(gv)


def test_kernel_support_and_symmetry():
    b = kernel.beta(6, 2.0)
    u = np.linspace(-3.5, 3.5, 141)
    v = kernel.phi(u, 6, b)
    assert np.all(v[np.abs(u) > 3] == 0)
    assert np.allclose(v, v[::-1], rtol=1e-14)
    assert abs(kernel.phi(np.array([3.0]), 6, b)[0] - 1.0) < 1e-15   # I0(0)


def test_fine_size():
    assert [kernel.fine_size(n, 2.0, 6) for n in (32, 128, 160, 192, 224)] == \
        [64, 256, 320, 384, 448]
    assert kernel.fine_size(11, 2.0, 6) == 24          # 22 = 2*11 is not smooth
    assert kernel.fine_size(3, 2.0, 6) == 12           # at least 2W
    for n in range(1, 200):
        m = kernel.fine_size(n, 2.0, 6)
        assert m % 2 == 0 and m >= 2 * n and kernel._smooth(m)


# ---------------------------------------------------------------- gridding
@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 10, 14), (9, 11, 7)])
def test_gridding_matches_direct(shape):
    g = np.random.default_rng(9)
    f = _img(shape, 10)
    k = g.uniform(-np.pi, np.pi, (2000, 3)).astype(np.float32)
    c = g.standard_normal(2000) + 1j * g.standard_normal(2000)
    op = gridding.Grid(shape)
    c2 = op.type2(f, k)
    ref2 = nudft.type2(f, k)
    assert np.linalg.norm(c2 - ref2) / np.linalg.norm(ref2) < 2e-5
    f1 = op.type1(c, k)
    ref1 = nudft.type1(c, k, shape)
    assert np.linalg.norm(f1 - ref1) / np.linalg.norm(ref1) < 2e-5


def test_gridding_accuracy_improves_with_width():
    shape = (10, 10, 10)
    g = np.random.default_rng(11)
    f = _img(shape, 12)
    k = g.uniform(-np.pi, np.pi, (800, 3))
    ref = nudft.type2(f, k)
    err = [np.linalg.norm(gridding.Grid(shape, 2.0, W).type2(f, k) - ref)
           / np.linalg.norm(ref) for W in (4, 6, 8)]
    assert err[0] > 5 * err[1] > 25 * err[2]


def test_gridding_on_grid_points_and_boundary_coordinates():
    # points exactly on fine-grid nodes, at k = 0 and at -pi (s - W/2 integer:
    # the half-open node rule decides which W nodes are used)
    shape = (8, 8, 8)
    f = _img(shape, 13)
    k = np.array([[0, 0, 0], [-np.pi, 0, 0], [-np.pi, -np.pi, -np.pi],
                  [np.pi / 2, -np.pi / 4, np.pi / 8]])
    ref = nudft.type2(f, k)
    got = gridding.type2(f, k)
    assert np.max(np.abs(got - ref)) < 5e-5 * np.max(np.abs(ref))


def test_gridding_adjoint_identity():
    shape = (10, 12, 9)
    op = gridding.Grid(shape)
    g = np.random.default_rng(14)
    f = _img(shape, 15)
    k = g.uniform(-np.pi, np.pi, (1500, 3))
    c = g.standard_normal(1500) + 1j * g.standard_normal(1500)
    lhs = np.vdot(c, op.type2(f, k))
    rhs = np.vdot(op.type1(c, k), f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gridding_stage_adjoints():
    # interp is the adjoint of spread, ifft*n the adjoint of fft, crop of pad
    shape = (6, 8, 10)
    op = gridding.Grid(shape)
    g = np.random.default_rng(16)
    G = _img(op.nf, 17)
    k = g.uniform(-np.pi, np.pi, (400, 3))
    c = g.standard_normal(400) + 1j * g.standard_normal(400)
    assert abs(np.vdot(c, op.interp(G, k)) - np.vdot(op.spread(c, k), G)) \
        < 1e-12 * np.linalg.norm(c) * np.linalg.norm(op.spread(c, k))
    H = _img(op.nf, 18)
    assert abs(np.vdot(H, op.fft(G)) - np.vdot(op.ifft(H), G)) \
        < 1e-10 * np.linalg.norm(H) * np.linalg.norm(G)
    f = _img(shape, 19)
    assert abs(np.vdot(H, op.deapodise_pad(f)) - np.vdot(op.crop_deapodise(H), f)) \
        < 1e-12 * np.linalg.norm(H) * np.linalg.norm(f)


def test_gridding_nodes_half_open():
    op = gridding.Grid((8, 8, 8))
    # s = k nf / 2pi: k = 0 gives s = 0, s - W/2 = -3 exactly -> nodes -2..3
    l0, w = op.nodes(np.zeros((1, 3)))
    assert np.all(l0 == -2)
    b = kernel.beta(6, 2.0)
    assert np.allclose(w[0, 0], kernel.phi(np.arange(2, -4, -1.0), 6, b))


# ---------------------------------------------------------------- MRF operator
def _mrf_case(shape=(6, 5, 4), K=2, C=3, B=2, T=4, M=60, seed=20):
    g = np.random.default_rng(seed)
    x = _img((K,) + shape, seed + 1)
    smaps = _img((C,) + shape, seed + 2)
    V = _img((T, K), seed + 3)
    frame = g.integers(0, T, M)
    k = g.uniform(-np.pi, np.pi, (M, 3))
    coil_idx = g.permutation(C)[:B]
    return x, smaps, coil_idx, V, frame, k


@pytest.mark.parametrize("kind,tol", [("direct", 1e-12), ("gridding", 2e-5)])
def test_mrf_forward_vs_frame_expansion(kind, tol):
    x, smaps, ci, V, frame, k = _mrf_case()
    op = mrf.Nufft(x.shape[1:], kind)
    y = mrf.forward(op, x, smaps, ci, V, frame, k)
    ref = mrf.forward_frames(x, smaps, ci, V, frame, k)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < tol


@pytest.mark.parametrize("kind", ["direct", "gridding"])
def test_mrf_adjoint_identity(kind):
    x, smaps, ci, V, frame, k = _mrf_case(seed=30)
    op = mrf.Nufft(x.shape[1:], kind)
    r = _img((len(ci), k.shape[0]), 31)
    lhs = np.vdot(r, mrf.forward(op, x, smaps, ci, V, frame, k))
    rhs = np.vdot(mrf.adjoint(op, r, smaps, ci, V, frame, k, x.shape[0]), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_mrf_reduces_to_plain_nufft():
    shape = (5, 6, 7)
    g = np.random.default_rng(40)
    f = _img(shape, 41)
    k = g.uniform(-np.pi, np.pi, (50, 3))
    op = mrf.Nufft(shape, "direct")
    y = mrf.forward(op, f[None], np.ones((1,) + shape), [0], np.ones((3, 1)),
                    g.integers(0, 3, 50), k)
    assert np.allclose(y[0], nudft.type2(f, k), atol=1e-12)


def test_normal_operator_full_cartesian():
    # T = 1, K = 1, |V| = 1, sum_c |S_c|^2 = 1 and every on-grid point once:
    # sum_c A_c^H A_c = N_vox * I
    shape = (4, 6, 5)
    C = 3
    S = _img((C,) + shape, 50)
    S /= np.sqrt(np.sum(np.abs(S) ** 2, axis=0))[None]
    k = _on_grid_points(shape)
    V = np.array([[np.exp(0.7j)]])
    frame = np.zeros(k.shape[0], dtype=np.int64)
    x = _img((1,) + shape, 51)
    op = mrf.Nufft(shape, "direct")
    y = mrf.forward(op, x, S, list(range(C)), V, frame, k)
    xb = mrf.adjoint(op, y, S, list(range(C)), V, frame, k, 1)
    assert np.allclose(xb, np.prod(shape) * x, rtol=1e-11, atol=1e-10)


@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_is_exact_central_difference(weighted):
    x, smaps, ci, V, frame, k = _mrf_case(seed=60)
    op = mrf.Nufft(x.shape[1:], "direct")
    d = _img((len(ci), k.shape[0]), 61)
    w = np.random.default_rng(62).uniform(0.2, 2.0, k.shape[0]) if weighted else None
    gr = mrf.dc_grad(op, x, smaps, ci, V, frame, k, d, w)
    for seed in (63, 64):
        dx = _img(x.shape, seed)
        for eps in (1e-1, 1.0):
            lp = mrf.dc_loss(op, x + eps * dx, smaps, ci, V, frame, k, d, w)
            lm = mrf.dc_loss(op, x - eps * dx, smaps, ci, V, frame, k, d, w)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - np.real(np.vdot(gr, dx))) < 1e-10 * abs(fd)
