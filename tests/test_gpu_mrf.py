"""Batched MRF subspace operator, adjoint, DC gradient and autograd through
the C ABI against the FP64 oracle (GPU), at sizes the oracle finishes in
seconds that still span many tiles and ragged tails."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import TOL, c64, host, rel, to_gpu
from oracle import mrf as omrf

pytestmark = pytest.mark.gpu


def _case(shape=(20, 18, 16), K=3, C=5, B=2, T=7, L=4, S=700, seed=3):
    traj, frame = wl.spiral_trajectory(T, L, S)
    x = wl.phantom(shape, K, seed, blur=0.7) + 0.1 * wl.random_image((K,) + shape, seed)
    smaps = wl.coil_maps(shape, C, seed)
    V = wl.subspace_basis(T, K, seed)
    ci = wl.coil_minibatch(C, B, seed)
    return dict(shape=shape, K=K, C=C, B=B, T=T, traj=traj, frame=frame, x=x.astype(np.complex64),
                smaps=smaps, V=V, coil_idx=ci)


def _gpu(c, **kw):
    p = sdn.Plan(to_gpu(c["traj"]), c["shape"], frame_of_point=to_gpu(c["frame"]), T=c["T"], **kw)
    return p, c64(c["x"]), c64(c["smaps"]), c64(c["V"])


@pytest.fixture(scope="module")
def case():
    return _case()


@pytest.fixture(scope="module")
def oracle_fwd(case):
    c = case
    op = omrf.Nufft(c["shape"], "direct")
    return omrf.forward(op, c["x"], c["smaps"], c["coil_idx"], c["V"], c["frame"], c["traj"])


def test_mrf_forward_vs_oracle(case, oracle_fwd):
    p, x, s, V = _gpu(case)
    y = host(sdn.mrf_forward(p, x, s, case["coil_idx"], V))
    assert rel(y, oracle_fwd) < TOL
    g = omrf.Nufft(case["shape"], "gridding")
    yg = omrf.forward(g, case["x"], case["smaps"], case["coil_idx"], case["V"], case["frame"],
                      case["traj"])
    assert rel(y, yg) < 5e-6
    for b in range(case["B"]):
        assert rel(y[b], oracle_fwd[b]) < TOL


def test_mrf_adjoint_vs_oracle(case):
    c = case
    p, x, s, V = _gpu(c)
    r = wl.random_kspace((c["B"], c["traj"].shape[0]), 21)
    xb = host(sdn.mrf_adjoint(p, c64(r), s, c["coil_idx"], V))
    op = omrf.Nufft(c["shape"], "direct")
    ref = omrf.adjoint(op, r, c["smaps"], c["coil_idx"], c["V"], c["frame"], c["traj"], c["K"])
    assert rel(xb, ref) < TOL
    for k in range(c["K"]):
        assert rel(xb[k], ref[k]) < TOL


def test_mrf_adjoint_identity_fp32(case):
    c = case
    p, x, s, V = _gpu(c)
    r = wl.random_kspace((c["B"], c["traj"].shape[0]), 22)
    y = host(sdn.mrf_forward(p, x, s, c["coil_idx"], V)).astype(np.complex128)
    xb = host(sdn.mrf_adjoint(p, c64(r), s, c["coil_idx"], V)).astype(np.complex128)
    lhs, rhs = np.vdot(r, y), np.vdot(xb, c["x"])
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


def test_batched_equals_plain_path(case):
    c = case
    p, x, s, V = _gpu(c)
    yb = host(sdn.mrf_forward(p, x, s, c["coil_idx"], V))
    yp = host(sdn.mrf_forward(p, x, s, c["coil_idx"], V, plain=True))
    assert rel(yb, yp) < 1e-6
    r = c64(wl.random_kspace((c["B"], c["traj"].shape[0]), 23))
    ab = host(sdn.mrf_adjoint(p, r, s, c["coil_idx"], V))
    ap = host(sdn.mrf_adjoint(p, r, s, c["coil_idx"], V, plain=True))
    assert rel(ab, ap) < 1e-6


def test_adjoint_accumulate(case):
    c = case
    p, x, s, V = _gpu(c)
    r = c64(wl.random_kspace((c["B"], c["traj"].shape[0]), 24))
    base = c64(wl.random_image((c["K"],) + c["shape"], 25))
    once = host(sdn.mrf_adjoint(p, r, s, c["coil_idx"], V))
    acc = host(sdn.mrf_adjoint(p, r, s, c["coil_idx"], V, out=base.clone(), accumulate=True))
    assert rel(acc, host(base) + once) < 1e-6


@pytest.mark.parametrize("weighted", [False, True])
def test_dc_loss_and_gradient_vs_oracle(case, oracle_fwd, weighted):
    c = case
    p, x, s, V = _gpu(c)
    M = c["traj"].shape[0]
    d = (oracle_fwd * 1.1 + 0.05 * wl.random_kspace((c["B"], M), 26)).astype(np.complex64)
    w = np.random.default_rng(27).uniform(0.2, 2.0, M).astype(np.float32) if weighted else None
    loss, grad = sdn.mrf_dc_grad(p, x, s, c["coil_idx"], V, c64(d),
                                 w=to_gpu(w) if weighted else None)
    op = omrf.Nufft(c["shape"], "direct")
    ref_l = omrf.dc_loss(op, c["x"], c["smaps"], c["coil_idx"], c["V"], c["frame"], c["traj"], d, w)
    ref_g = omrf.dc_grad(op, c["x"], c["smaps"], c["coil_idx"], c["V"], c["frame"], c["traj"], d, w)
    assert abs(host(loss)[0] - ref_l) / ref_l < 1e-4
    assert rel(host(grad), ref_g) < TOL


def test_autograd_backward_is_the_adjoint(case, oracle_fwd):
    c = case
    p, x, s, V = _gpu(c)
    M = c["traj"].shape[0]
    d = c64((oracle_fwd * 0.9).astype(np.complex64))
    xr = x.clone().requires_grad_(True)
    y = sdn.MRFForward.apply(xr, p, s, c["coil_idx"], V)
    loss = torch.sum(torch.abs(y - d) ** 2)
    loss.backward()
    l2, g2 = sdn.mrf_dc_grad(p, x, s, c["coil_idx"], V, d)
    assert rel(host(xr.grad), host(g2)) < 1e-5
    assert abs(loss.item() - host(l2)[0]) / host(l2)[0] < 1e-5
    op = omrf.Nufft(c["shape"], "direct")
    ref_g = omrf.dc_grad(op, c["x"], c["smaps"], c["coil_idx"], c["V"], c["frame"], c["traj"],
                         host(d), None)
    assert rel(host(xr.grad), ref_g) < TOL


def test_autograd_directional_derivative(case, oracle_fwd):
    # the loss is quadratic: the central difference equals Re<g, dx> exactly.
    # d is kept well away from A x so the residual is not rounding noise.
    c = case
    p, x, s, V = _gpu(c)
    M = c["traj"].shape[0]
    d = c64((0.6 * oracle_fwd + 0.3 * wl.random_kspace((c["B"], M), 30)).astype(np.complex64))
    dx = c64(wl.random_image((c["K"],) + c["shape"], 28))
    _, g = sdn.mrf_dc_grad(p, x, s, c["coil_idx"], V, d)
    eps = 0.05
    lp, _ = sdn.mrf_dc_grad(p, x + eps * dx, s, c["coil_idx"], V, d)
    lm, _ = sdn.mrf_dc_grad(p, x - eps * dx, s, c["coil_idx"], V, d)
    fd = (host(lp)[0] - host(lm)[0]) / (2 * eps)
    an = float(np.real(np.vdot(host(g).astype(np.complex128), host(dx).astype(np.complex128))))
    assert abs(fd - an) / abs(an) < 1e-4


def test_budgeted_coil_chunks_equal_one_pass(case):
    c = case
    p, x, s, V = _gpu(c)
    nf = p.info()["fine"]
    one_coil = int(np.prod(nf)) * c["K"] * 8
    q, _, _, _ = _gpu(c, workspace_budget=one_coil)
    y1 = host(sdn.mrf_forward(p, x, s, c["coil_idx"], V))
    y2 = host(sdn.mrf_forward(q, x, s, c["coil_idx"], V))
    assert rel(y2, y1) < 1e-6
    r = c64(wl.random_kspace((c["B"], c["traj"].shape[0]), 29))
    assert rel(host(sdn.mrf_adjoint(q, r, s, c["coil_idx"], V)),
               host(sdn.mrf_adjoint(p, r, s, c["coil_idx"], V))) < 1e-6
    with pytest.raises(sdn.SdnError) as e:
        small, _, _, _ = _gpu(c, workspace_budget=one_coil // 2)
        sdn.mrf_forward(small, x, s, c["coil_idx"], V)
    assert e.value.status == -3


def test_argument_errors(case):
    c = case
    p, x, s, V = _gpu(c)
    with pytest.raises(sdn.SdnError) as e:
        sdn.mrf_forward(p, x, s, [0, c["C"]], V)
    assert e.value.status == -2
    with pytest.raises(sdn.SdnError) as e:
        sdn.mrf_forward(p, x, s, [0, -1], V)
    assert e.value.status == -2
    p.close()
    with pytest.raises(sdn.SdnError):
        sdn.mrf_forward(p, x, s, [0], V)


def test_point_orders_agree(case, oracle_fwd):
    """Every tile in cell order gives the same per-point sums (bit for bit:
    a point's interpolation does not depend on its neighbours' order) and
    the same adjoint up to the summation order; the library rejects an
    unknown order."""
    c = case
    p, x, s, V = _gpu(c)
    q, _, _, _ = _gpu(c, point_order="cell")
    y0 = host(sdn.mrf_forward(p, x, s, c["coil_idx"], V))
    y1 = host(sdn.mrf_forward(q, x, s, c["coil_idx"], V))
    assert np.array_equal(y0, y1)
    assert rel(y1, oracle_fwd) < TOL
    r = c64(wl.random_kspace((c["B"], c["traj"].shape[0]), 33))
    assert rel(host(sdn.mrf_adjoint(q, r, s, c["coil_idx"], V)),
               host(sdn.mrf_adjoint(p, r, s, c["coil_idx"], V))) < 1e-6
    o = sdn.Opts()
    sdn.lib().sdn_default_opts(ctypes.byref(o))
    o.point_order = 7
    h = ctypes.c_void_p()
    t = to_gpu(c["traj"])
    st = sdn.lib().sdn_plan_create(ctypes.byref(h), (ctypes.c_int64 * 3)(*c["shape"]),
                                   ctypes.c_void_p(t.data_ptr()), int(t.shape[0]), None, 1,
                                   ctypes.byref(o), None)
    assert st == -1 and not h.value   # SDN_E_INVALID


@pytest.mark.parametrize("B", [8, 16, 6])
def test_adjoint_coil_counts_of_the_fused_inverse_x_pass(B):
    """8 and 16 coils take the inverse x pass fused with the coil sum (2 and 1
    image rows per workgroup), 6 the separate crop and sum; all equal the
    plain per-coil/per-channel path and the FP64 oracle."""
    shape, K, T = (12, 14, 16), 2, 3
    traj, frame = wl.spiral_trajectory(T, 4, 200)
    p = sdn.Plan(to_gpu(traj), shape, frame_of_point=to_gpu(frame), T=T)
    smaps = wl.coil_maps(shape, B, 31)
    V = wl.subspace_basis(T, K, 31)
    ci = np.arange(B, dtype=np.int32)[::-1].copy()
    r = wl.random_kspace((B, traj.shape[0]), 32)
    ab = host(sdn.mrf_adjoint(p, c64(r), c64(smaps), ci, c64(V)))
    ap = host(sdn.mrf_adjoint(p, c64(r), c64(smaps), ci, c64(V), plain=True))
    assert rel(ab, ap) < 1e-6
    ref = omrf.adjoint(omrf.Nufft(shape, "gridding"), r, smaps, ci, V, frame,
                       traj.astype(np.float64), K)
    assert rel(ab, ref) < 2e-5

