"""Helpers shared by the GPU tests (not a test module)."""

import numpy as np
import torch

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
