"""Total-variation penalty on the TSMI and its gradient, FP64.

Test infrastructure only.

Alg. 1 adds lambda TV(x_hat) to the per-coil loss (the StoDIP + TV variant
of Sec. 2.2).  The paper does not define the TV form; the reading taken
here is the isotropic TV over the three spatial axes, per subspace
channel, with forward differences that are zero at the last index of an
axis (Neumann boundary) and a smoothing eps > 0 that keeps it
differentiable where the image is flat:

    TV(x) = sum_k sum_n t_k[n],
    t_k[n] = sqrt(|D_x x_k[n]|^2 + |D_y x_k[n]|^2 + |D_z x_k[n]|^2 + eps^2),
    D_d x[n] = x[n + e_d] - x[n] when n_d + 1 < N_d, else 0.

Its gradient in PyTorch's complex convention (dTV/dRe x + i dTV/dIm x) is
the transpose of the differences applied to q_d = D_d x / t:

    g[m] = sum_d (q_d[m - e_d] - q_d[m]),   q_d[m - e_d] = 0 when m_d = 0.

x is [K, Nz, Ny, Nx]; axis d of the image is array axis 3 (x), 2 (y), 1 (z).
"""

import numpy as np

_AXES = (3, 2, 1)   # x, y, z


def differences(x):
    """[D_x x, D_y x, D_z x], each shaped like x."""
    x = np.asarray(x, dtype=np.complex128)
    out = []
    for ax in _AXES:
        d = np.zeros_like(x)
        n = x.shape[ax]
        hi = [slice(None)] * 4
        lo = [slice(None)] * 4
        hi[ax] = slice(1, n)
        lo[ax] = slice(0, n - 1)
        d[tuple(lo)] = x[tuple(hi)] - x[tuple(lo)]
        out.append(d)
    return out


def magnitude(x, eps):
    """t[k, z, y, x] of the definition."""
    return np.sqrt(sum(np.abs(d) ** 2 for d in differences(x)) + float(eps) ** 2)


def value(x, eps):
    return float(np.sum(magnitude(x, eps)))


def grad(x, eps):
    t = magnitude(x, eps)
    g = np.zeros(np.shape(x), dtype=np.complex128)
    for ax, d in zip(_AXES, differences(x)):
        q = d / t
        n = q.shape[ax]
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        g -= q
        g[tuple(hi)] += q[tuple(lo)]
    return g
