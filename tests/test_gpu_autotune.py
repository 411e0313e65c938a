"""Autotuner on the GPU: it returns a runnable option set, and a plan built
with it gives the DC gradient of the default plan (engines agree to ~4e-7)."""

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import c64, to_gpu

pytestmark = pytest.mark.gpu


def test_autotune_result_is_valid_and_cached(tmp_path):
    shape, K, C, B, T = (32, 32, 32), 3, 4, 2, 10
    traj, frame = wl.spiral_trajectory(T, 8, 512)
    cache = str(tmp_path / "tune.json")
    best = sdn.autotune(to_gpu(traj), shape, B, K, frame_of_point=to_gpu(frame), T=T, cache=cache)
    assert best["tile"] in (0, 8, 16) and best["max_points_per_item"] in (0, 1024)
    assert best["spread_engine"] in ("gather", "matrix", "planes") and best["ms"] > 0
    assert best["point_order"] in ("auto", "cell")
    assert best["point_order"] == "auto" or best["spread_engine"] == "gather"
    assert sdn.autotune(to_gpu(traj), shape, B, K, frame_of_point=to_gpu(frame), T=T,
                        cache=cache) == best
    x = c64(wl.phantom(shape, K, 3, blur=1.0))
    smaps = c64(wl.coil_maps(shape, C, 3))
    V = c64(wl.subspace_basis(T, K, 3))
    ci = np.array([0, 2], dtype=np.int32)
    d = c64(wl.random_kspace((B, traj.shape[0]), 4))
    opts = {k: best[k] for k in sdn.TUNED_KEYS}
    pt = sdn.Plan(to_gpu(traj), shape, frame_of_point=to_gpu(frame), T=T, **opts)
    p0 = sdn.Plan(to_gpu(traj), shape, frame_of_point=to_gpu(frame), T=T)
    l1, g1 = sdn.mrf_dc_grad(pt, x, smaps, ci, V, d)
    l0, g0 = sdn.mrf_dc_grad(p0, x, smaps, ci, V, d)
    assert (torch.linalg.norm(g1 - g0) / torch.linalg.norm(g0)).item() < 2e-6
    assert abs(l1.item() - l0.item()) <= 1e-6 * abs(l0.item())
