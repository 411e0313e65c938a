"""Helpers shared by the GPU tests (not a test module)."""

import numpy as np
import torch

from oracle import nudft

TOL = 1e-4          # relative l2 bound of the HIP FP32 path against the FP64 oracle


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_gpu(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def c64(a):
    return to_gpu(np.asarray(a, dtype=np.complex64))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def uniform_points(M, seed):
    g = np.random.default_rng(seed)
    return g.uniform(-np.pi, np.pi, (M, 3)).astype(np.float32)


def cimg(shape, seed):
    g = np.random.default_rng(seed)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)


def direct_forward_at(w, idx):
    """y_b(j) for the sampled points j, from the definitions (direct NUDFT)."""
    x, S, V = w["x"], w["smaps"], w["V"]
    k = w["traj"][idx]
    t = w["frame"][idx]
    y = np.zeros((len(w["coil_idx"]), len(idx)), dtype=np.complex128)
    for b, c in enumerate(w["coil_idx"]):
        for kk in range(x.shape[0]):
            y[b] += V[t, kk] * nudft.type2(S[c].astype(np.complex128) * x[kk], k, chunk=len(idx))
    return y


def direct_adjoint_at(w, r, sel, chunk=200000):
    """xbar_k at a Cartesian product of voxels, from the definitions."""
    k = w["traj"].astype(np.float64)
    V = w["V"].astype(np.complex128)
    t = w["frame"]
    shape = w["shape"]
    mz, my, mx = (nudft.modes(n)[np.asarray(s)] for n, s in zip(shape, sel))
    K = V.shape[1]
    B = r.shape[0]
    acc = np.zeros((B, K, len(mz), len(my), len(mx)), dtype=np.complex128)
    for a in range(0, k.shape[0], chunk):
        b_ = min(k.shape[0], a + chunk)
        ex = np.exp(1j * np.outer(k[a:b_, 0], mx))
        ey = np.exp(1j * np.outer(k[a:b_, 1], my))
        ez = np.exp(1j * np.outer(k[a:b_, 2], mz))
        E = (ez[:, :, None, None] * ey[:, None, :, None] * ex[:, None, None, :]).reshape(b_ - a, -1)
        cv = np.conj(V[t[a:b_]])                                   # [m, K]
        for b in range(B):
            coef = cv * r[b, a:b_, None]                            # [m, K]
            acc[b] += (coef.T @ E).reshape(K, len(mz), len(my), len(mx))
    out = np.zeros((K, len(mz), len(my), len(mx)), dtype=np.complex128)
    for b, c in enumerate(w["coil_idx"]):
        sc = np.conj(w["smaps"][c][np.ix_(*sel)].astype(np.complex128))
        out += sc[None] * acc[b]
    return out
