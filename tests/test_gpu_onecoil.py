"""The one-coil step of Algorithm 1 (one coil per stochastic update) and the
vector-ALU gather spreading with the subspace mix (GPU).

A call with a single coil spreads through the gather engine with the mix
fused in (one wave per spreading block, K channels in registers); the
matrix-core engine serves calls of several coils unless the plan forces the
gather.  These tests run that engine at K = 5, 6 and 8 (one coil, as the
paper's step and the paper-shaped benchmark row do) and forced at several
coils, against the FP64 oracle: the direct NUDFT (<= 1e-4 relative l2) and
the FP64 gridding NUFFT with the same kernel (<= 5e-6).
"""

import numpy as np
import pytest

import paper_2408_02367_amd as sdn
import workloads as wl
from gpu_common import TOL, c64, host, rel, to_gpu
from oracle import mrf as omrf

pytestmark = pytest.mark.gpu


def _case(K, B, shape=(20, 18, 16), C=6, T=7, L=4, S=700, seed=41):
    traj, frame = wl.spiral_trajectory(T, L, S)
    x = (wl.phantom(shape, K, seed, blur=0.7)
         + 0.1 * wl.random_image((K,) + shape, seed)).astype(np.complex64)
    return dict(shape=shape, K=K, B=B, T=T, traj=traj, frame=frame, x=x,
                smaps=wl.coil_maps(shape, C, seed), V=wl.subspace_basis(T, K, seed),
                coil_idx=wl.coil_minibatch(C, B, seed))


def _plan(c, **kw):
    return sdn.Plan(to_gpu(c["traj"]), c["shape"], frame_of_point=to_gpu(c["frame"]), T=c["T"],
                    **kw)


def _check_grad_and_adjoint(c, p):
    M = c["traj"].shape[0]
    x, s, V = c64(c["x"]), c64(c["smaps"]), c64(c["V"])
    direct = omrf.Nufft(c["shape"], "direct")
    grid = omrf.Nufft(c["shape"], "gridding")
    args = (c["smaps"], c["coil_idx"], c["V"], c["frame"], c["traj"])
    y_ref = omrf.forward(direct, c["x"], *args)
    d = (0.7 * y_ref + 0.2 * wl.random_kspace((c["B"], M), 42)).astype(np.complex64)
    loss, g = sdn.mrf_dc_grad(p, x, s, c["coil_idx"], V, c64(d))
    g = host(g)
    ref_l = omrf.dc_loss(direct, c["x"], *args, d)
    assert abs(host(loss)[0] - ref_l) / ref_l < TOL
    assert rel(g, omrf.dc_grad(direct, c["x"], *args, d)) < TOL
    assert rel(g, omrf.dc_grad(grid, c["x"], *args, d)) < 5e-6
    r = wl.random_kspace((c["B"], M), 43)
    xb = host(sdn.mrf_adjoint(p, c64(r), s, c["coil_idx"], V))
    assert rel(xb, omrf.adjoint(direct, r, c["smaps"], c["coil_idx"], c["V"], c["frame"],
                                c["traj"], c["K"])) < TOL
    ref_g = omrf.adjoint(grid, r, c["smaps"], c["coil_idx"], c["V"], c["frame"], c["traj"], c["K"])
    assert rel(xb, ref_g) < 5e-6
    for k in range(c["K"]):
        assert rel(xb[k], ref_g[k]) < 5e-6


@pytest.mark.parametrize("K", [5, 6, 8])
def test_one_coil_gradient_and_adjoint(K):
    c = _case(K, 1, T=max(7, K + 2))
    _check_grad_and_adjoint(c, _plan(c))


@pytest.mark.parametrize("K", [5, 6])
def test_one_coil_cell_order(K):
    """The plan option that orders every interpolation tile by first cell
    (faster for the one-coil gather) gives the same operator."""
    c = _case(K, 1, seed=44)
    _check_grad_and_adjoint(c, _plan(c, point_order="cell"))


@pytest.mark.parametrize("K,B", [(5, 2), (6, 3), (4, 4)])
def test_gather_engine_forced_at_several_coils(K, B):
    c = _case(K, B, seed=45 + K)
    p = _plan(c, spread_engine="gather")
    assert p.spread_engine(B, K) == "gather"
    _check_grad_and_adjoint(c, p)
    # and it equals both matrix-core engines to the FP32 summation order
    r = c64(wl.random_kspace((B, c["traj"].shape[0]), 46))
    s, V = c64(c["smaps"]), c64(c["V"])
    ref = host(sdn.mrf_adjoint(p, r, s, c["coil_idx"], V))
    for engine in ("matrix", "planes"):
        q = _plan(c, spread_engine=engine)
        assert q.spread_engine(B, K) == engine
        assert rel(host(sdn.mrf_adjoint(q, r, s, c["coil_idx"], V)), ref) < 1e-6, engine


@pytest.mark.parametrize("K,B", [(6, 8), (5, 4), (2, 3), (8, 7), (3, 20)])
def test_plane_split_engine(K, B):
    """The plane-split matrix spreading (the automatic choice from 32 coil-
    channel pairs) against the oracle, at column tilings of 1 to 6 tiles
    and several coil groups per block (K = 3, B = 20: two groups)."""
    c = _case(K, B, C=max(B, 6), T=max(7, K + 2), seed=50 + K + B)
    p = _plan(c, spread_engine="planes")
    assert p.spread_engine(B, K) == "planes"
    _check_grad_and_adjoint(c, p)
    if K * B >= 32:
        assert _plan(c).spread_engine(B, K) == "planes"


@pytest.mark.parametrize("engine", ["planes", "matrix"])
def test_matrix_engines_ragged_blocks(engine):
    """Both matrix-core engines on fine grids that 8-cell blocks do not
    divide on any axis (36 x 42 x 50 cells: the last block of each axis is
    cut), so their write-out of cell pairs meets every edge, against the
    oracle."""
    c = _case(5, 4, shape=(18, 21, 25), C=6, T=7, seed=61)
    p = _plan(c, spread_engine=engine)
    assert p.spread_engine(4, 5) == engine
    _check_grad_and_adjoint(c, p)
