"""Type-2 / type-1 NUFFTs on grids whose axes use the compile-time FFT
lengths 96, 160, 224, 288 and 400 (400 = the paper's 200^3 volume at
sigma = 2), against the direct NUDFT at sampled points and voxels."""

import numpy as np
import pytest

import paper_2408_02367_amd as sdn
from gpu_common import c64, cimg, host, rel, to_gpu, uniform_points
from oracle import nudft

pytestmark = pytest.mark.gpu

# the W = 6, sigma = 2 gridding NUFFT itself is ~1e-5 from the exact NUDFT in
# 3D; a wrong FFT pass would be off by O(1)
TOL_DIRECT = 5e-5


# (Nz, Ny, Nx) -> fine (2 Nz, 2 Ny, 2 Nx): the x pass and both strided passes
@pytest.mark.parametrize("shape", [(48, 80, 200), (144, 112, 112), (16, 200, 48)])
def test_specialised_lengths_match_direct(shape):
    M = 4000
    k = uniform_points(M, 11)
    p = sdn.Plan(to_gpu(k), shape)
    assert tuple(p.info()["fine"]) == tuple(2 * n for n in shape)
    f = cimg(shape, 12)
    c = host(p.forward(c64(f[None]))[0])
    idx = np.random.default_rng(13).choice(M, 24, replace=False)
    ref = nudft.type2(f.astype(np.complex128), k[idx].astype(np.float64), chunk=24)
    assert rel(c[idx], ref) < TOL_DIRECT
    cc = cimg((M,), 14)
    img = host(p.adjoint(c64(cc[None]))[0])
    g = np.random.default_rng(15)
    sel = tuple(np.sort(g.choice(n, 3, replace=False)) for n in shape)
    ref1 = nudft.type1(cc.astype(np.complex128), k.astype(np.float64), shape, sel=sel)
    assert rel(img[np.ix_(*sel)], ref1) < TOL_DIRECT


def test_plan_with_records_above_two_gib_matches_direct():
    """29M points: the transposed per-point records exceed 2 GiB, so the
    interpolation reads them with plain global loads instead of buffer loads."""
    import torch
    M, shape = 29_000_000, (24, 20, 16)
    g = torch.Generator(device="cuda").manual_seed(21)
    k = (torch.rand(M, 3, generator=g, device="cuda") * (2 * np.pi) - np.pi).contiguous()
    p = sdn.Plan(k, shape)
    assert M * (3 * 6 + 1) * 4 > 2 ** 31
    f = cimg(shape, 22)
    c = p.forward(c64(f[None]))[0]
    idx = np.random.default_rng(23).choice(M, 24, replace=False)
    kk = host(k[torch.from_numpy(idx).cuda()]).astype(np.float64)
    ref = nudft.type2(f.astype(np.complex128), kk, chunk=24)
    assert rel(host(c[torch.from_numpy(idx).cuda()]), ref) < TOL_DIRECT
    del c, p
    torch.cuda.synchronize()
