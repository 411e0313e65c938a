"""The DC gradient without allocation against sdn_mrf_dc_grad (GPU).

sdn_mrf_dc_grad_noalloc keeps its buffers in a static device array of the
library instead of the plan's workspace.  Called through the C ABI, it must
return what sdn_mrf_dc_grad returns: bit for bit when both take all coils in
one pass, to the FP32 summation order when the static array forces coil
passes.  Two calls in a row, the second smaller, check that nothing of the
first call's contents leaks into the second.
"""

import ctypes

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import c64, to_gpu

pytestmark = pytest.mark.gpu

LIMIT = 64 << 20


def _lib():
    return sdn.lib()


def _case(shape, K, C, B, T, L, S, seed):
    traj, frame = wl.spiral_trajectory(T, L, S)
    p = sdn.Plan(to_gpu(traj), shape, frame_of_point=to_gpu(frame), T=T)
    x = c64(wl.phantom(shape, K, seed, blur=0.8) + 0.1 * wl.random_image((K,) + shape, seed))
    s = c64(wl.coil_maps(shape, C, seed))
    V = c64(wl.subspace_basis(T, K, seed))
    ci = wl.coil_minibatch(C, B, seed)
    d = c64(wl.random_kspace((B, traj.shape[0]), seed + 1))
    return p, x, s, V, ci, d


def _noalloc(p, x, s, ci, V, d):
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    grad = torch.full_like(x, float("nan"))
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=x.device)
    st = _lib().sdn_mrf_dc_grad_noalloc(
        p.handle, ctypes.c_void_p(x.data_ptr()), x.shape[0], ctypes.c_void_p(s.data_ptr()),
        s.shape[0], ci.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(ci),
        ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(d.data_ptr()), None,
        ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, loss, grad


def test_two_calls_in_a_row_equal_the_allocating_entry_point():
    # the second call is smaller (shape, points, coils, channels) than the first
    cases = [((24, 20, 28), 5, 8, 4, 9, 6, 900, 71), ((16, 18, 12), 3, 5, 2, 4, 3, 500, 72)]
    for shape, K, C, B, T, L, S, seed in cases:
        p, x, s, V, ci, d = _case(shape, K, C, B, T, L, S, seed)
        assert p.workspace_size(B, K) < LIMIT       # one pass: same launches, same bits
        st, loss, grad = _noalloc(p, x, s, ci, V, d)
        assert st == 0, sdn.lib().sdn_last_error().decode()
        l_ref, g_ref = sdn.mrf_dc_grad(p, x, s, ci, V, d)
        torch.cuda.synchronize()
        assert torch.equal(loss, l_ref) and torch.equal(grad, g_ref), shape


def test_plane_split_spreading_without_allocation():
    # 8 coils x 6 channels: the plane-split matrix-core spreading; then a
    # smaller call with the one-wave-per-coil engine
    cases = [((16, 16, 16), 6, 10, 8, 9, 2, 300, 75), ((16, 14, 18), 4, 5, 3, 6, 3, 400, 76)]
    for (shape, K, C, B, T, L, S, seed), engine in zip(cases, ("planes", "matrix")):
        p, x, s, V, ci, d = _case(shape, K, C, B, T, L, S, seed)
        assert p.spread_engine(B, K) == engine
        assert p.workspace_size(B, K) < LIMIT
        st, loss, grad = _noalloc(p, x, s, ci, V, d)
        assert st == 0, sdn.lib().sdn_last_error().decode()
        l_ref, g_ref = sdn.mrf_dc_grad(p, x, s, ci, V, d)
        torch.cuda.synchronize()
        assert torch.equal(loss, l_ref) and torch.equal(grad, g_ref), shape


def test_coil_passes_when_the_static_array_is_too_small_for_all_coils():
    # 80^3 fine grids: 4 MiB per channel, 5 channels per coil, 4 coils do not fit
    p, x, s, V, ci, d = _case((40, 40, 40), 5, 6, 4, 6, 8, 800, 73)
    assert p.workspace_size(4, 5) > LIMIT > p.workspace_size(1, 5)
    st, loss, grad = _noalloc(p, x, s, ci, V, d)
    assert st == 0, sdn.lib().sdn_last_error().decode()
    l_ref, g_ref = sdn.mrf_dc_grad(p, x, s, ci, V, d)
    assert (torch.linalg.norm(grad - g_ref) / torch.linalg.norm(g_ref)).item() < 1e-6
    assert abs(loss.item() - l_ref.item()) <= 1e-12 * l_ref.item()
    # and again, smaller: a plan of one pass after the call of several
    p2, x2, s2, V2, ci2, d2 = _case((12, 14, 16), 2, 3, 2, 3, 2, 300, 74)
    st, loss2, grad2 = _noalloc(p2, x2, s2, ci2, V2, d2)
    assert st == 0
    l2, g2 = sdn.mrf_dc_grad(p2, x2, s2, ci2, V2, d2)
    torch.cuda.synchronize()
    assert torch.equal(loss2, l2) and torch.equal(grad2, g2)


def test_too_large_for_the_static_array_is_an_error():
    # 192^3 fine grids: one coil's 5 channels alone take 283 MB
    p, x, s, V, ci, d = _case((96, 96, 96), 5, 2, 1, 2, 2, 300, 75)
    st, _, _ = _noalloc(p, x, s, ci, V, d)
    assert st == -3   # SDN_E_NOMEM
    assert b"static workspace" in sdn.lib().sdn_last_error()
