"""Parity at the large batched size (GPU): 224^3 x K = 6, a minibatch of 8 of
48 coils, T = 1200 frames x 12 interleaves x 1400 samples (M = 20.16M),
W = 6, sigma = 2 (448^3 fine grids, 34.5 GB for the 48 channels).

Outputs at seeded random points (forward) and voxels (adjoint) against the
direct NUDFT computed one by one; the memory-budgeted (coil-chunked) DC
gradient against the unbudgeted one; the DC gradient against the exact
central difference of the loss.
"""

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import TOL, c64, direct_adjoint_at, direct_forward_at, host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c5():
    w = wl.make("c5", minibatch_maps=True)
    dev = torch.device("cuda", 0)
    traj = torch.from_numpy(w["traj"]).to(dev)
    frame = torch.from_numpy(w["frame"]).to(dev)
    plan = sdn.Plan(traj, w["shape"], frame_of_point=frame, T=w["T"])
    return dict(w=w, plan=plan, traj=traj, frame=frame, x=c64(w["x"]), s=c64(w["smaps"]),
                ci=w["coil_idx"], V=c64(w["V"]))


def test_c5_forward_sampled_points(c5):
    w, p = c5["w"], c5["plan"]
    y = host(sdn.mrf_forward(p, c5["x"], c5["s"], c5["ci"], c5["V"]))
    M = w["traj"].shape[0]
    idx = np.sort(np.random.default_rng(51).choice(M, 16, replace=False))
    idx = np.unique(np.concatenate([idx, np.arange(0, M, 1400)[:8]]))   # k-space centre too
    assert rel(y[:, idx], direct_forward_at(w, idx)) < TOL


def test_c5_adjoint_sampled_voxels(c5):
    w, p = c5["w"], c5["plan"]
    B, M = len(c5["ci"]), w["traj"].shape[0]
    r = wl.random_kspace((B, M), 52)
    xb = host(sdn.mrf_adjoint(p, c64(r), c5["s"], c5["ci"], c5["V"]))
    sel = ([7, 150], [100, 223], [0, 111])
    assert rel(xb[(slice(None),) + np.ix_(*sel)], direct_adjoint_at(w, r, sel)) < TOL


def test_c5_budgeted_chunks_match_and_gradient_is_exact(c5):
    w, p = c5["w"], c5["plan"]
    B, M = len(c5["ci"]), w["traj"].shape[0]
    d = c64(wl.random_kspace((B, M), 53))
    l_full, g_full = sdn.mrf_dc_grad(p, c5["x"], c5["s"], c5["ci"], c5["V"], d)
    # 12 GB of fine-grid workspace: two coils (12 channels of 448^3) per pass
    pb = sdn.Plan(c5["traj"], w["shape"], frame_of_point=c5["frame"], T=w["T"],
                  workspace_budget=12 << 30)
    l_b, g_b = sdn.mrf_dc_grad(pb, c5["x"], c5["s"], c5["ci"], c5["V"], d)
    assert (torch.linalg.norm(g_b - g_full) / torch.linalg.norm(g_full)).item() < 1e-6
    assert abs(l_b.item() - l_full.item()) <= 1e-6 * abs(l_full.item())
    assert pb.workspace_size(B, w["K"]) <= (12 << 30) + (1 << 30)
    del pb
    # the loss is quadratic: the central difference is its exact derivative
    # for any step; a larger step keeps L(x+) - L(x-) well above the FP32
    # rounding of two losses of this size (~1e13)
    dx = c64(wl.random_image((w["K"],) + w["shape"], 54))
    eps = 0.5
    lp, _ = sdn.mrf_dc_grad(p, c5["x"] + eps * dx, c5["s"], c5["ci"], c5["V"], d)
    lm, _ = sdn.mrf_dc_grad(p, c5["x"] - eps * dx, c5["s"], c5["ci"], c5["V"], d)
    fd = (lp.item() - lm.item()) / (2 * eps)
    an = torch.vdot(g_full.flatten().to(torch.complex128), dx.flatten().to(torch.complex128)).real.item()
    assert abs(fd - an) / abs(an) < 1e-4
