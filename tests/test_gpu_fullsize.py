"""Parity on the production fine-grid lengths and at the benchmarked size (GPU).

* shapes whose fine grids use the compile-time FFT passes (64 ... 448),
  including odd image sizes, against the direct NUDFT;
* the batched MRF operator on a 32^3 image (64^3 grid) against the oracle;
* the benchmarked workload - 160^3 x K = 5, a 4-coil minibatch of 32,
  T = 1000 frames x 8 interleaves x 1200 samples (M = 9.6M), W = 6,
  sigma = 2 - in the launch configuration the benchmark times: outputs at
  seeded random points (forward) and voxels (adjoint) against the direct
  NUDFT computed one by one; one (coil, channel) type 2 and type 1 over
  the whole output array against the FP64 gridding oracle; the autograd
  gradient of the DC loss (d = A x_true + 1% noise from the FP64 oracle,
  x a 10% smooth perturbation of x_true) against the fused DC gradient and
  against 2 A^H (A x - d) from the oracle at sampled voxels; plus
  properties that hold at any size.
"""

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import (TOL, c64, cimg, direct_adjoint_at, direct_forward_at, host, rel, to_gpu,
                        uniform_points)
from oracle import cloops, gridding, nudft
from oracle import mrf as omrf

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(31, 95, 64), (96, 32, 128), (24, 40, 160)])
def test_compile_time_lengths_vs_direct(shape):
    M = 6000
    traj = uniform_points(M, 40 + shape[0])
    f = cimg(shape, 41)
    p = sdn.Plan(to_gpu(traj), shape)
    nf = p.info()["fine"]
    assert nf == tuple(gridding.Grid(shape).nf)
    y = host(p.forward(c64(f[None])))[0]
    assert rel(y, nudft.type2(f, traj)) < TOL
    c = cimg((M,), 42)
    sel = ([0, shape[0] // 2, shape[0] - 1], [1, shape[1] // 3, shape[1] - 2],
           list(range(0, shape[2], max(1, shape[2] // 7))))
    img = host(p.adjoint(c64(c[None])))[0]
    ref = nudft.type1(c, traj, shape, sel=sel)
    assert rel(img[np.ix_(*sel)], ref) < TOL
    g = gridding.Grid(shape)
    assert rel(img, g.type1(c, traj)) < 5e-6


def test_batched_mrf_32cubed_vs_oracle():
    shape, K, C, B, T = (32, 32, 32), 5, 8, 4, 10
    traj, frame = wl.spiral_trajectory(T, 8, 512)
    x = wl.phantom(shape, K, 7, blur=1.0).astype(np.complex64)
    smaps = wl.coil_maps(shape, C, 7)
    V = wl.subspace_basis(T, K, 7)
    ci = wl.coil_minibatch(C, B, 7)
    p = sdn.Plan(to_gpu(traj), shape, frame_of_point=to_gpu(frame), T=T)
    y = host(sdn.mrf_forward(p, c64(x), c64(smaps), ci, c64(V)))
    op = omrf.Nufft(shape, "gridding")
    ref = omrf.forward(op, x, smaps, ci, V, frame, traj)
    assert rel(y, ref) < 5e-6
    sub = np.random.default_rng(8).choice(traj.shape[0], 300, replace=False)
    dop = omrf.Nufft(shape, "direct")
    refd = omrf.forward(dop, x, smaps, ci, V, frame[sub], traj[sub])
    assert rel(y[:, sub], refd) < TOL
    r = wl.random_kspace((B, traj.shape[0]), 9)
    xb = host(sdn.mrf_adjoint(p, c64(r), c64(smaps), ci, c64(V)))
    assert rel(xb, omrf.adjoint(op, r, smaps, ci, V, frame, traj, K)) < 5e-6


# ------------------------------------------------------------ benchmarked size
@pytest.fixture(scope="module")
def big():
    w = wl.make("c4")
    dev = torch.device("cuda", 0)
    plan = sdn.Plan(torch.from_numpy(w["traj"]).to(dev), w["shape"],
                    frame_of_point=torch.from_numpy(w["frame"]).to(dev), T=w["T"])
    ci = w["coil_idx"]
    return dict(w=w, plan=plan, x=c64(w["x"]), s=c64(w["smaps"][ci]),
                ci_local=np.arange(len(ci), dtype=np.int32), V=c64(w["V"]))


def test_benchmark_size_forward_sampled_points(big):
    w, p = big["w"], big["plan"]
    y = host(sdn.mrf_forward(p, big["x"], big["s"], big["ci_local"], big["V"]))
    idx = np.sort(np.random.default_rng(11).choice(w["traj"].shape[0], 96, replace=False))
    # the k-space centre is the hottest tile: sample it too
    idx = np.unique(np.concatenate([idx, np.arange(0, 9600000, 1200)[:32]]))
    ref = direct_forward_at(w, idx)
    assert rel(y[:, idx], ref) < TOL


def test_benchmark_size_adjoint_sampled_voxels(big):
    w, p = big["w"], big["plan"]
    B, M = len(w["coil_idx"]), w["traj"].shape[0]
    r = wl.random_kspace((B, M), 12)
    xb = host(sdn.mrf_adjoint(p, c64(r), big["s"], big["ci_local"], big["V"]))
    sel = ([20, 80, 131], [3, 79, 150], [0, 64, 80, 159])
    ref = direct_adjoint_at(w, r, sel)
    assert rel(xb[(slice(None),) + np.ix_(*sel)], ref) < TOL


def test_benchmark_size_adjoint_identity_and_batched_vs_plain(big):
    w, p = big["w"], big["plan"]
    B, M = len(w["coil_idx"]), w["traj"].shape[0]
    r = c64(wl.random_kspace((B, M), 13))
    y = sdn.mrf_forward(p, big["x"], big["s"], big["ci_local"], big["V"])
    xb = sdn.mrf_adjoint(p, r, big["s"], big["ci_local"], big["V"])
    lhs = torch.vdot(r.flatten().to(torch.complex128), y.flatten().to(torch.complex128))
    rhs = torch.vdot(xb.flatten().to(torch.complex128), big["x"].flatten().to(torch.complex128))
    assert abs((lhs - rhs) / lhs).item() < 1e-5
    yp = sdn.mrf_forward(p, big["x"], big["s"], big["ci_local"], big["V"], plain=True)
    assert (torch.linalg.norm(yp - y) / torch.linalg.norm(y)).item() < 1e-6
    xp = sdn.mrf_adjoint(p, r, big["s"], big["ci_local"], big["V"], plain=True)
    assert (torch.linalg.norm(xp - xb) / torch.linalg.norm(xb)).item() < 1e-6


def test_benchmark_size_dc_gradient_is_exact_directional_derivative(big):
    w, p = big["w"], big["plan"]
    B, M = len(w["coil_idx"]), w["traj"].shape[0]
    d = c64(wl.random_kspace((B, M), 14))
    dx = c64(wl.random_image((w["K"],) + w["shape"], 15))
    _, g = sdn.mrf_dc_grad(p, big["x"], big["s"], big["ci_local"], big["V"], d)
    eps = 0.05
    lp, _ = sdn.mrf_dc_grad(p, big["x"] + eps * dx, big["s"], big["ci_local"], big["V"], d)
    lm, _ = sdn.mrf_dc_grad(p, big["x"] - eps * dx, big["s"], big["ci_local"], big["V"], d)
    fd = (lp.item() - lm.item()) / (2 * eps)
    an = torch.vdot(g.flatten().to(torch.complex128), dx.flatten().to(torch.complex128)).real.item()
    assert abs(fd - an) / abs(an) < 1e-4


@pytest.fixture(scope="module")
def big_nodes(big):
    """The FP64 oracle's kernel nodes of the 9.6M benchmark points."""
    g = gridding.Grid(big["w"]["shape"])
    return g, cloops.node_chunks(g, big["w"]["traj"])


def test_benchmark_size_type2_full_array_vs_gridding(big, big_nodes):
    """One (coil, channel) of the benchmark: plain type 2 of S_c x_k at all
    9.6M points against the FP64 gridding NUFFT with the same kernel."""
    w, p = big["w"], big["plan"]
    g, nodes = big_nodes
    f = (w["smaps"][w["coil_idx"][0]] * w["x"][0]).astype(np.complex64)
    y = host(p.forward(c64(f[None])))[0]
    ref = cloops.interp_many(g, g.fft(g.deapodise_pad(f.astype(np.complex128))), w["traj"],
                             nodes=nodes)[0]
    assert rel(y, ref) < 5e-6
    # the k-space centre (the densest tiles) on its own
    centre = np.arange(0, w["traj"].shape[0], 1200)
    assert rel(y[centre], ref[centre]) < 5e-6


def test_benchmark_size_type1_full_array_vs_gridding(big, big_nodes):
    """Plain type 1 of one row of random k-space values at all 9.6M points,
    compared over the whole 160^3 image."""
    w, p = big["w"], big["plan"]
    g, nodes = big_nodes
    r = wl.random_kspace((1, w["traj"].shape[0]), 16)
    img = host(p.adjoint(c64(r)))[0]
    ref = g.crop_deapodise(g.ifft(cloops.spread_many(g, r, w["traj"], nodes=nodes)[0]))
    assert rel(img, ref) < 5e-6


def test_benchmark_size_autograd_gradient_vs_oracle(big, big_nodes):
    """MRFForward + loss.backward() at the benchmark size: equal to the fused
    DC gradient, and to the oracle's 2 A^H (A x - d) at sampled voxels, with
    d = A x_true + 1% complex noise made by the FP64 oracle and x = x_true +
    a smooth perturbation of 10% RMS (so |A x - d| is about 0.1 |d|)."""
    w, p = big["w"], big["plan"]
    g, nodes = big_nodes
    shape, K = w["shape"], w["K"]
    ci = w["coil_idx"]
    B, M = len(ci), w["traj"].shape[0]
    x_true = w["x"].astype(np.complex64)
    pert = wl.phantom(shape, K, w["seed"] + 100)
    pert *= 0.1 * np.sqrt(np.mean(np.abs(x_true) ** 2) / np.mean(np.abs(pert) ** 2))
    x = (x_true + pert).astype(np.complex64)
    V = w["V"].astype(np.complex128)
    Vt = V[w["frame"]]                                         # [M, K]

    def oracle_forward(img):
        y = np.zeros((B, M), dtype=np.complex128)
        for b, c in enumerate(ci):
            S = w["smaps"][c].astype(np.complex128)
            Gs = np.stack([g.fft(g.deapodise_pad(S * img[k].astype(np.complex128)))
                           for k in range(K)])
            u = cloops.interp_many(g, Gs, w["traj"], nodes=nodes)
            del Gs
            y[b] = np.sum(Vt.T * u, axis=0)
        return y

    y_true = oracle_forward(x_true)
    rms = np.sqrt(np.mean(np.abs(y_true) ** 2, axis=1))
    d = (y_true + wl.complex_noise((B, M), 0.01, rms, w["seed"])).astype(np.complex64)
    r = oracle_forward(x) - d.astype(np.complex128)
    assert 0.03 < np.linalg.norm(r) / np.linalg.norm(d) < 0.3

    xr = c64(x).requires_grad_(True)
    dd = c64(d)
    y = sdn.MRFForward.apply(xr, p, big["s"], big["ci_local"], big["V"])
    loss = torch.sum(torch.view_as_real(y - dd).double() ** 2)
    loss.backward()
    l_dc, g_dc = sdn.mrf_dc_grad(p, c64(x), big["s"], big["ci_local"], big["V"], dd)
    assert rel(host(xr.grad), host(g_dc)) < 1e-6
    assert abs(loss.item() - l_dc.item()) <= 1e-6 * l_dc.item()
    l_ref = float(np.sum(np.abs(r) ** 2))
    assert abs(l_dc.item() - l_ref) <= 1e-4 * l_ref

    sel = ([5, 40, 81, 120, 158], [2, 77, 80, 141], [0, 33, 80, 112, 159])
    ref = 2.0 * direct_adjoint_at(w, r, sel)
    gs = host(g_dc)[(slice(None),) + np.ix_(*sel)]
    assert rel(gs, ref) < TOL
