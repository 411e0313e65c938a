"""The DC loss and gradient are bitwise repeatable (GPU).

Every sum of the DC step has a fixed order: interpolation sums a point's
cells in a fixed order, the loss adds per-workgroup partials in two
fixed-order levels (no atomics), spreading walks each block's sorted list,
and the inverse x pass adds the coils in order.  Two calls, and replays of a
captured step, must therefore return identical bits.
"""

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import c64, to_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("B,engine", [(4, "auto"), (1, "auto"), (3, "gather"), (7, "planes")])
def test_dc_step_is_bitwise_repeatable(B, engine):
    shape, K, C, T = (24, 20, 28), 5, 8, 9
    traj, frame = wl.spiral_trajectory(T, 6, 900)
    p = sdn.Plan(to_gpu(traj), shape, frame_of_point=to_gpu(frame), T=T, spread_engine=engine)
    x = c64(wl.phantom(shape, K, 61, blur=0.8))
    s = c64(wl.coil_maps(shape, C, 61))
    V = c64(wl.subspace_basis(T, K, 61))
    ci = wl.coil_minibatch(C, B, 61)
    d = c64(wl.random_kspace((B, traj.shape[0]), 62))
    l1, g1 = sdn.mrf_dc_grad(p, x, s, ci, V, d)
    l1, g1 = l1.clone(), g1.clone()
    l2, g2 = sdn.mrf_dc_grad(p, x, s, ci, V, d)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)
    # replays of the captured step, with eager work between them
    grad = torch.empty_like(x)
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sdn.mrf_dc_grad(p, x, s, ci, V, d, grad=grad, loss=loss)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sdn.mrf_dc_grad(p, x, s, ci, V, d, grad=grad, loss=loss)
    for i in range(3):
        grad.zero_()
        loss.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(loss, l1) and torch.equal(grad, g1), f"replay {i}"
        sdn.mrf_dc_grad(p, x + 1.0, s, ci, V, d)   # eager work between replays
        torch.cuda.synchronize()
