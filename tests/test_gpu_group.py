"""Ragged volumes through one group call (GPU): 128^3, 160^3 and
192 x 192 x 160 images, each with its own spiral trajectory (T = 512, 1000,
1440 frames x 8 interleaves x 1200 samples) and basis, K = 5, a 4-coil
minibatch of 32 each (P = 20 per volume).

The group must equal the member plans called one by one; one volume is also
checked against the direct NUDFT at sampled points.
"""

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import TOL, c64, direct_forward_at, host, rel

pytestmark = pytest.mark.gpu

VOLUMES = ("c3r128", "c4", "c3r192")


@pytest.fixture(scope="module")
def ragged():
    dev = torch.device("cuda", 0)
    ws, plans = [], []
    for name in VOLUMES:
        w = wl.make(name, minibatch_maps=True)
        ws.append(w)
        plans.append(sdn.Plan(torch.from_numpy(w["traj"]).to(dev), w["shape"],
                              frame_of_point=torch.from_numpy(w["frame"]).to(dev), T=w["T"]))
    args = dict(x=[c64(w["x"]) for w in ws], smaps=[c64(w["smaps"]) for w in ws],
                coil_idx=[w["coil_idx"] for w in ws], V=[c64(w["V"]) for w in ws])
    return ws, plans, sdn.PlanGroup(plans), args


def test_group_equals_member_plans(ragged):
    ws, plans, group, a = ragged
    ys = group.mrf_forward(a["x"], a["smaps"], a["coil_idx"], a["V"])
    for v, p in enumerate(plans):
        ref = sdn.mrf_forward(p, a["x"][v], a["smaps"][v], a["coil_idx"][v], a["V"][v])
        assert torch.equal(ys[v], ref)
    d = [c64(wl.random_kspace((4, p.M), 60 + v)) for v, p in enumerate(plans)]
    loss, grads = group.mrf_dc_grad(a["x"], a["smaps"], a["coil_idx"], a["V"], d)
    total = 0.0
    for v, p in enumerate(plans):
        l1, g1 = sdn.mrf_dc_grad(p, a["x"][v], a["smaps"][v], a["coil_idx"][v], a["V"][v], d[v])
        assert torch.equal(grads[v], g1)
        total += l1.item()
    assert abs(loss.item() - total) <= 1e-12 * abs(total)
    xs = group.mrf_adjoint(d, a["smaps"], a["coil_idx"], a["V"])
    for v, p in enumerate(plans):
        assert torch.equal(xs[v], sdn.mrf_adjoint(p, d[v], a["smaps"][v], a["coil_idx"][v], a["V"][v]))


def test_group_volume_vs_direct(ragged):
    ws, plans, group, a = ragged
    ys = group.mrf_forward(a["x"], a["smaps"], a["coil_idx"], a["V"])
    w = ws[2]                                   # 192 x 192 x 160
    M = w["traj"].shape[0]
    idx = np.sort(np.random.default_rng(61).choice(M, 24, replace=False))
    assert rel(host(ys[2])[:, idx], direct_forward_at(w, idx)) < TOL


def test_group_argument_errors(ragged):
    ws, plans, group, a = ragged
    with pytest.raises(ValueError):
        group.mrf_forward(a["x"][:2], a["smaps"], a["coil_idx"], a["V"])
    bad = [np.arange(3, dtype=np.int32), a["coil_idx"][1], a["coil_idx"][2]]
    with pytest.raises(ValueError):
        group.mrf_forward(a["x"], a["smaps"], bad, a["V"])


def _small_group(K, B, shapes=((20, 18, 16), (24, 20, 28), (16, 16, 16)), W=(6, 6, 6), seed=70,
                 **kw):
    dev = torch.device("cuda", 0)
    plans, args = [], dict(x=[], smaps=[], coil_idx=[], V=[], d=[])
    C = max(B, 6)
    for v, shape in enumerate(shapes):
        T = K + 2 + v
        traj, frame = wl.spiral_trajectory(T, 3, 400 + 100 * v)
        plans.append(sdn.Plan(torch.from_numpy(traj).to(dev), shape, W=W[v],
                              frame_of_point=torch.from_numpy(frame).to(dev), T=T, **kw))
        args["x"].append(c64(wl.phantom(shape, K, seed + v, blur=0.7)
                             + 0.1 * wl.random_image((K,) + shape, seed + v)))
        args["smaps"].append(c64(wl.coil_maps(shape, C, seed + v)))
        args["coil_idx"].append(wl.coil_minibatch(C, B, seed + v))
        args["V"].append(c64(wl.subspace_basis(T, K, seed + v)))
        args["d"].append(c64(wl.random_kspace((B, traj.shape[0]), seed + 10 + v)))
    return plans, args


def _interp_launches(plans):
    return [p.profile_read(reset=True).get("interp", (0.0, 0))[1] for p in plans]


@pytest.mark.parametrize("K,B,engine", [(5, 4, "matrix"), (6, 8, "planes"), (5, 1, "gather")])
def test_fused_group_equals_member_plans(K, B, engine):
    """One interpolation and one spreading launch for all volumes (seen in
    the first plan's stage events) give the member plans' results bit for
    bit: the same work items run the same arithmetic."""
    plans, a = _small_group(K, B)
    assert all(p.spread_engine(B, K) == engine for p in plans)
    group = sdn.PlanGroup(plans)
    for p in plans:
        p.profile(True)
        p.profile_read(reset=True)
    loss, grads = group.mrf_dc_grad(a["x"], a["smaps"], a["coil_idx"], a["V"], a["d"])
    torch.cuda.synchronize()
    assert _interp_launches(plans) == [1, 0, 0]
    total = 0.0
    for v, p in enumerate(plans):
        l1, g1 = sdn.mrf_dc_grad(p, a["x"][v], a["smaps"][v], a["coil_idx"][v], a["V"][v],
                                 a["d"][v])
        assert torch.equal(grads[v], g1), v
        total += l1.item()
    assert abs(loss.item() - total) <= 1e-12 * abs(total)
    ys = group.mrf_forward(a["x"], a["smaps"], a["coil_idx"], a["V"])
    xs = group.mrf_adjoint(a["d"], a["smaps"], a["coil_idx"], a["V"])
    for v, p in enumerate(plans):
        assert torch.equal(ys[v], sdn.mrf_forward(p, a["x"][v], a["smaps"][v], a["coil_idx"][v],
                                                  a["V"][v]))
        assert torch.equal(xs[v], sdn.mrf_adjoint(p, a["d"][v], a["smaps"][v], a["coil_idx"][v],
                                                  a["V"][v]))
    for p in plans:
        p.profile(False)


@pytest.mark.parametrize("case", ["widths", "budget"])
def test_group_falls_back_to_member_calls(case):
    """Volumes that cannot share launches (different kernel widths; a budget
    that splits the minibatch into coil passes) run member by member, with
    the same results."""
    K, B = 3, 4
    if case == "widths":
        plans, a = _small_group(K, B, W=(6, 4, 6))
    else:
        # two coils of the largest volume per pass: that volume runs in coil passes
        plans, a = _small_group(K, B, workspace_budget=48 * 40 * 56 * K * 8 * 2)
    group = sdn.PlanGroup(plans)
    for p in plans:
        p.profile(True)
        p.profile_read(reset=True)
    loss, grads = group.mrf_dc_grad(a["x"], a["smaps"], a["coil_idx"], a["V"], a["d"])
    torch.cuda.synchronize()
    launches = _interp_launches(plans)
    assert launches[1] >= 1 and launches[2] >= 1
    for v, p in enumerate(plans):
        _, g1 = sdn.mrf_dc_grad(p, a["x"][v], a["smaps"][v], a["coil_idx"][v], a["V"][v],
                                a["d"][v])
        assert torch.equal(grads[v], g1), v
    for p in plans:
        p.profile(False)
