"""Pipe-Menon density compensation on the GPU against the FP64 oracle."""

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import host, rel, to_gpu
from oracle import dcf, gridding

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,iters", [((14, 16, 12), 1), ((14, 16, 12), 6), ((20, 18, 24), 4)])
def test_dcf_matches_oracle(shape, iters):
    traj, _ = wl.spiral_trajectory(5, 6, 350)
    p = sdn.Plan(to_gpu(traj), shape)
    w = host(sdn.dcf_estimate(p, iters))
    ref = dcf.pipe_menon(gridding.Grid(shape), traj.astype(np.float64), iters)
    assert rel(w, ref) < 2e-5


def test_dcf_shifted_full_grid_is_the_closed_form_constant():
    shape = (8, 8, 8)
    g = gridding.Grid(shape)
    nf = g.nf[0]
    m = np.arange(nf) + 0.5
    kz, ky, kx = np.meshgrid(m, m, m, indexing="ij")
    k = (2 * np.pi * np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1) / nf).astype(np.float32)
    w = host(sdn.dcf_estimate(sdn.Plan(to_gpu(k), shape), 3))
    ref = dcf.pipe_menon(g, k.astype(np.float64), 3)
    assert rel(w, ref) < 1e-5
    assert np.ptp(w) <= 1e-5 * np.abs(w).max()


def test_dcf_weighted_gradient_uses_the_estimate():
    shape, K, C, B, T = (16, 16, 16), 2, 3, 2, 4
    traj, frame = wl.spiral_trajectory(T, 6, 300)
    p = sdn.Plan(to_gpu(traj), shape, frame_of_point=to_gpu(frame), T=T)
    w = sdn.dcf_estimate(p, 5)
    x = to_gpu(wl.phantom(shape, K, 9, blur=1.0).astype(np.complex64))
    smaps = to_gpu(wl.coil_maps(shape, C, 9))
    V = to_gpu(wl.subspace_basis(T, K, 9))
    d = to_gpu(wl.random_kspace((B, traj.shape[0]), 10).astype(np.complex64))
    ci = np.array([0, 2], dtype=np.int32)
    l_w, g_w = sdn.mrf_dc_grad(p, x, smaps, ci, V, d, w=w)
    y = sdn.mrf_forward(p, x, smaps, ci, V)
    r = (y - d) * w[None, :]
    ref_l = torch.sum(w[None, :].double() * torch.abs(y - d).double() ** 2).item()
    ref_g = 2 * sdn.mrf_adjoint(p, r.contiguous(), smaps, ci, V)
    assert abs(l_w.item() - ref_l) <= 1e-5 * ref_l
    assert (torch.linalg.norm(g_w - ref_g) / torch.linalg.norm(ref_g)).item() < 1e-5
