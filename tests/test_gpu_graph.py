"""The batched DC step captured in a HIP graph (GPU).

After one eager call has sized the plan's workspace, a call enqueues only
kernels on the caller's stream (no allocation, no memset, no host sync), so
torch.cuda.graph can capture it. Every replay is checked against the eager
result, with eager work and synchronisations between the replays.
"""

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import c64, to_gpu

pytestmark = pytest.mark.gpu


def _problem():
    shape, K, C, B, T = (24, 20, 22), 4, 6, 3, 9
    traj, frame = wl.spiral_trajectory(T, 6, 400)
    x = wl.phantom(shape, K, 21, blur=1.0).astype(np.complex64)
    smaps = wl.coil_maps(shape, C, 21)
    V = wl.subspace_basis(T, K, 21)
    ci = wl.coil_minibatch(C, B, 21)
    d = wl.random_kspace((B, traj.shape[0]), 22)
    p = sdn.Plan(to_gpu(traj), shape, frame_of_point=to_gpu(frame), T=T)
    return p, c64(x), c64(smaps), ci, c64(V), c64(d)


def test_dc_gradient_graph_replays_match_eager():
    p, x, smaps, ci, V, d = _problem()
    grad = torch.empty_like(x)
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    ref_loss, ref_grad = sdn.mrf_dc_grad(p, x, smaps, ci, V, d)   # also sizes the workspace
    torch.cuda.synchronize()
    ref_loss, ref_grad = ref_loss.clone(), ref_grad.clone()

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        sdn.mrf_dc_grad(p, x, smaps, ci, V, d, grad=grad, loss=loss)   # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        sdn.mrf_dc_grad(p, x, smaps, ci, V, d, grad=grad, loss=loss)

    for rep in range(4):
        grad.zero_()
        loss.zero_()
        g.replay()
        torch.cuda.synchronize()
        err = (torch.linalg.norm(grad - ref_grad) / torch.linalg.norm(ref_grad)).item()
        assert err < 1e-6, (rep, err)
        assert abs(loss.item() - ref_loss.item()) <= 1e-6 * abs(ref_loss.item()), rep
        # eager work on the same plan between replays
        l2, g2 = sdn.mrf_dc_grad(p, x, smaps, ci, V, d)
        torch.cuda.synchronize()
        assert (torch.linalg.norm(g2 - ref_grad) / torch.linalg.norm(ref_grad)).item() < 1e-6


def test_forward_graph_with_new_inputs_each_replay():
    p, x, smaps, ci, V, _ = _problem()
    y = sdn.mrf_forward(p, x, smaps, ci, V)
    torch.cuda.synchronize()
    xin = x.clone()
    out = torch.empty_like(y)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sdn.mrf_forward(p, xin, smaps, ci, V, out=out)
    gen = torch.Generator(device="cuda").manual_seed(5)
    for rep in range(3):
        xin.copy_(torch.randn(x.shape, dtype=torch.complex64, device=x.device, generator=gen))
        g.replay()
        torch.cuda.synchronize()
        ref = sdn.mrf_forward(p, xin, smaps, ci, V)
        torch.cuda.synchronize()
        assert (torch.linalg.norm(out - ref) / torch.linalg.norm(ref)).item() < 1e-6, rep
