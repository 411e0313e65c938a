"""Initialisers (normal operator, conjugate gradients, scaled adjoint), the
full-coil DC gradient under a workspace budget and the TV penalty on the
GPU, against the FP64 oracle."""

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import c64, host, rel, to_gpu
from oracle import mrf, recon, tv

pytestmark = pytest.mark.gpu

SHAPE, K, C, T = (14, 16, 12), 3, 3, 4


def _problem(seed, shape=SHAPE, K=K, C=C, T=T, S=300):
    traj, frame = wl.spiral_trajectory(T, 6, S)
    M = traj.shape[0]
    g = np.random.default_rng(seed)
    return dict(
        traj=traj, frame=frame, shape=shape,
        x=wl.phantom(shape, K, seed, blur=1.0).astype(np.complex64),
        smaps=wl.coil_maps(shape, C, seed),
        V=wl.subspace_basis(T, K, seed),
        w=g.uniform(0.5, 1.5, M).astype(np.float32),
        y=wl.random_kspace((C, M), seed + 1).astype(np.complex64))


def _plan(P):
    return sdn.Plan(to_gpu(P["traj"]), P["shape"], frame_of_point=to_gpu(P["frame"]), T=T)


def _op(P):
    return mrf.Nufft(P["shape"], "gridding")


def _k(P):
    return P["traj"].astype(np.float64)


@pytest.mark.parametrize("lam", [0.0, 2.5])
def test_normal_operator_matches_oracle(lam):
    P = _problem(3)
    p = _plan(P)
    out = host(sdn.mrf_normal(p, c64(P["x"]), c64(P["smaps"]), c64(P["V"]),
                              w=to_gpu(P["w"]), lam=lam))
    ref = recon.normal(_op(P), P["x"], P["smaps"], P["V"], P["frame"], _k(P), P["w"], lam)
    assert rel(out, ref) < 2e-5


@pytest.mark.parametrize("lam,iters", [(0.0, 4), (1.0e3, 3)])
def test_cg_matches_oracle(lam, iters):
    P = _problem(5)
    p = _plan(P)
    x0 = 0.1 * P["x"]
    x, hist = sdn.mrf_cg(p, c64(P["y"]), c64(P["smaps"]), c64(P["V"]), x0=c64(x0),
                         iterations=iters, w=to_gpu(P["w"]), lam=lam)
    rx, rh = recon.cg(_op(P), P["y"], P["smaps"], P["V"], P["frame"], _k(P), x0, iters,
                      w=P["w"], lam=lam)
    assert rel(host(x), rx) < 1e-4
    h = host(hist)
    assert np.all(np.abs(h - rh) <= 1e-4 * np.abs(rh)), (h, rh)


def test_cg_zero_iterations_keeps_the_start_point():
    P = _problem(6)
    p = _plan(P)
    x0 = c64(P["x"])
    x, hist = sdn.mrf_cg(p, c64(P["y"]), c64(P["smaps"]), c64(P["V"]), x0=x0, iterations=0)
    assert torch.equal(x, x0)
    b = recon.rhs(_op(P), P["y"], P["smaps"], P["V"], P["frame"], _k(P), K)
    r = b - recon.normal(_op(P), P["x"], P["smaps"], P["V"], P["frame"], _k(P))
    assert abs(host(hist)[0] - np.vdot(r, r).real) <= 1e-4 * np.vdot(r, r).real


def test_cg_on_coil_subset_and_graph_replay():
    P = _problem(7)
    p = _plan(P)
    ci = np.array([2, 0], dtype=np.int32)
    y = c64(P["y"][ci])
    smaps, V = c64(P["smaps"]), c64(P["V"])
    ref_x, ref_h = sdn.mrf_cg(p, y, smaps, V, iterations=3, coil_idx=ci, K=K)
    torch.cuda.synchronize()
    ref_x, ref_h = ref_x.clone(), ref_h.clone()
    rx, _ = recon.cg(_op(P), P["y"][ci], P["smaps"][ci], P["V"], P["frame"], _k(P),
                     np.zeros((K,) + SHAPE), 3)
    assert rel(host(ref_x), rx) < 1e-4
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gx, gh = sdn.mrf_cg(p, y, smaps, V, iterations=3, coil_idx=ci, K=K)
    for rep in range(3):
        gx.fill_(7.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(gx, ref_x), rep
        assert torch.equal(gh, ref_h), rep
        sdn.mrf_normal(p, ref_x, smaps, V, coil_idx=ci)   # eager work on the plan between replays
        torch.cuda.synchronize()


def test_scaled_adjoint_matches_oracle():
    P = _problem(8)
    p = _plan(P)
    x, s = sdn.mrf_scaled_adjoint(p, c64(P["y"]), c64(P["smaps"]), c64(P["V"]), w=to_gpu(P["w"]))
    rx, rs = recon.scaled_adjoint(_op(P), P["y"], P["smaps"], P["V"], P["frame"], _k(P), K, P["w"])
    assert rel(host(x), rx) < 2e-5
    assert abs(host(s)[0] - rs) <= 2e-5 * rs


def test_full_coil_gradient_under_budget_equals_minibatch_sum():
    shape, Cf = (24, 20, 22), 8
    P = _problem(9, shape=shape, C=Cf)
    x, smaps, V = c64(P["x"]), c64(P["smaps"]), c64(P["V"])
    d = c64(P["y"])
    free = _plan(P)
    budget = free.workspace_size(2, K)            # two coils per pass
    tight = sdn.Plan(to_gpu(P["traj"]), shape, frame_of_point=to_gpu(P["frame"]), T=T,
                     workspace_budget=budget)
    allc = np.arange(Cf, dtype=np.int32)
    loss, grad = sdn.mrf_dc_grad(tight, x, smaps, allc, V, d)
    lsum, gsum = 0.0, torch.zeros_like(x)
    for b0 in range(0, Cf, 2):
        l, gr = sdn.mrf_dc_grad(free, x, smaps, allc[b0:b0 + 2], V, d[b0:b0 + 2])
        lsum += l.item()
        gsum += gr
    torch.cuda.synchronize()
    assert abs(loss.item() - lsum) <= 1e-9 * lsum
    assert rel(host(grad), host(gsum)) < 1e-6
    ref = mrf.dc_grad(_op(P), P["x"], P["smaps"], list(range(Cf)), P["V"], P["frame"], _k(P),
                      P["y"])
    assert rel(host(grad), ref) < 2e-5


@pytest.mark.parametrize("shape,Kt,eps", [(SHAPE, 3, 0.05), ((5, 7, 9), 1, 1e-3), ((1, 6, 33), 2, 0.2)])
def test_tv_matches_oracle(shape, Kt, eps):
    traj, _ = wl.spiral_trajectory(2, 4, 100)
    p = sdn.Plan(to_gpu(traj), shape)
    x = wl.phantom(shape, Kt, 4, blur=1.0).astype(np.complex64) if min(shape) > 2 else \
        (np.random.default_rng(4).standard_normal((Kt,) + shape)
         + 1j * np.random.default_rng(5).standard_normal((Kt,) + shape)).astype(np.complex64)
    lam = 0.7
    v, g = sdn.tv_grad(p, c64(x), eps, lam)
    assert abs(host(v)[0] - lam * tv.value(x, eps)) <= 1e-6 * lam * tv.value(x, eps)
    assert rel(host(g), lam * tv.grad(x, eps)) < 2e-5


def test_tv_accumulates_onto_a_gradient_and_flat_image():
    traj, _ = wl.spiral_trajectory(2, 4, 100)
    p = sdn.Plan(to_gpu(traj), SHAPE)
    x = c64(wl.phantom(SHAPE, 2, 6, blur=1.0))
    base = c64(np.random.default_rng(1).standard_normal((2,) + SHAPE))
    g = base.clone()
    v, g = sdn.tv_grad(p, x, 0.1, 2.0, grad=g, accumulate=True)
    _, g1 = sdn.tv_grad(p, x, 0.1, 2.0)
    torch.cuda.synchronize()
    assert rel(host(g), host(base + g1)) < 1e-6
    flat = torch.full((2,) + SHAPE, 0.3 - 0.1j, dtype=torch.complex64, device="cuda")
    v, gf = sdn.tv_grad(p, flat, 0.25, 1.5)
    n = 2 * np.prod(SHAPE)
    assert abs(host(v)[0] - 1.5 * 0.25 * n) <= 1e-6 * 1.5 * 0.25 * n
    assert torch.count_nonzero(gf).item() == 0
    vo, none = sdn.tv_grad(p, x, 0.1, 1.0, want_grad=False)
    assert none is None and abs(host(vo)[0] - tv.value(host(x), 0.1)) <= 1e-6 * host(vo)[0]


def test_recon_argument_errors():
    P = _problem(2)
    p = _plan(P)
    x = c64(P["x"])
    with pytest.raises(sdn.SdnError):
        sdn.tv_grad(p, x, 0.0)
    with pytest.raises(sdn.SdnError):
        sdn.tv_grad(p, x, float("nan"))
    with pytest.raises(sdn.SdnError):
        sdn.mrf_normal(p, x, c64(P["smaps"]), c64(P["V"]), lam=-1.0)
    with pytest.raises(sdn.SdnError):
        sdn.mrf_cg(p, c64(P["y"]), c64(P["smaps"]), c64(P["V"]), iterations=-1)
    with pytest.raises(ValueError):
        sdn.mrf_scaled_adjoint(p, c64(P["y"][:2]), c64(P["smaps"]), c64(P["V"]))
