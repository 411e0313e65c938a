"""MRF subspace forward operator, adjoint, DC loss and gradient in FP64.

Test infrastructure only.

Sec. 2 defines the forward operator A: C^{N x K} -> C^{C x M x L x T} as
coil sensitivities, a NUFFT and a temporal SVD (subspace) compression;
Eq. 3 splits the data-consistency loss over coils, A = {A_c}.  The reading
taken here (the paper does not spell out the composition): the TSMI x has K
subspace channels x_k; sample j of k-space belongs to timeframe t_j, whose
signal is the subspace expansion sum_k V[t_j, k] x_k, so for a minibatch of
coils c_b (b = 0..B-1)

    y_b(j) = sum_k V[t_j, k] NUFFT2(S_{c_b} * x_k)(k_j)              (A)
    xbar_k = sum_b conj(S_{c_b}) * NUFFT1(conj(V[t_j, k]) r_b(j))    (A^H)

The DC loss of Eq. 2-3 with a real weight w_j >= 0 (the DCF; 1 when absent)
and its gradient in PyTorch's complex convention (dL/dRe x + i dL/dIm x):

    L(x) = sum_b sum_j w_j |y_b(j) - d_b(j)|^2,     g = 2 A^H (w (A x - d))
"""

import numpy as np

from . import gridding, nudft


class Nufft:
    """Type-2 / type-1 NUFFT pair: the exact NUDFT or the FP64 gridding one."""

    def __init__(self, shape, kind="gridding", sigma=2.0, W=6):
        self.shape = tuple(shape)
        self.kind = kind
        if kind == "gridding":
            self.grid = gridding.Grid(self.shape, sigma, W)
        elif kind != "direct":
            raise ValueError(kind)

    def t2(self, f, k):
        if self.kind == "direct":
            return nudft.type2(f, k)
        return self.grid.type2(f, k)

    def t1(self, c, k):
        if self.kind == "direct":
            return nudft.type1(c, k, self.shape)
        return self.grid.type1(c, k)


def forward(op, x, smaps, coil_idx, V, frame, k):
    """y[b, j] for x[K, Nz, Ny, Nx], smaps[C, Nz, Ny, Nx], V[T, K]."""
    x = np.asarray(x, dtype=np.complex128)
    V = np.asarray(V, dtype=np.complex128)
    frame = np.asarray(frame)
    K = x.shape[0]
    y = np.zeros((len(coil_idx), np.shape(k)[0]), dtype=np.complex128)
    for b, c in enumerate(coil_idx):
        s = np.asarray(smaps[c], dtype=np.complex128)
        for kk in range(K):
            y[b] += V[frame, kk] * op.t2(s * x[kk], k)
    return y


def adjoint(op, r, smaps, coil_idx, V, frame, k, K):
    """xbar[K, Nz, Ny, Nx] = A^H r for r[B, M]."""
    r = np.asarray(r, dtype=np.complex128)
    V = np.asarray(V, dtype=np.complex128)
    frame = np.asarray(frame)
    xbar = np.zeros((K,) + op.shape, dtype=np.complex128)
    for b, c in enumerate(coil_idx):
        sc = np.conj(np.asarray(smaps[c], dtype=np.complex128))
        for kk in range(K):
            xbar[kk] += sc * op.t1(np.conj(V[frame, kk]) * r[b], k)
    return xbar


def dc_loss(op, x, smaps, coil_idx, V, frame, k, d, w=None):
    r = forward(op, x, smaps, coil_idx, V, frame, k) - np.asarray(d)
    ww = 1.0 if w is None else np.asarray(w, dtype=np.float64)[None, :]
    return float(np.sum(ww * np.abs(r) ** 2))


def dc_grad(op, x, smaps, coil_idx, V, frame, k, d, w=None):
    r = forward(op, x, smaps, coil_idx, V, frame, k) - np.asarray(d)
    if w is not None:
        r = r * np.asarray(w, dtype=np.float64)[None, :]
    return 2.0 * adjoint(op, r, smaps, coil_idx, V, frame, k, np.shape(x)[0])


def forward_frames(x, smaps, coil_idx, V, frame, k):
    """Brute force of (A) for tiny sizes: expand every frame image
    X_t = sum_k V[t, k] x_k, then take the exact NUDFT of S_{c_b} X_t at the
    points of frame t only."""
    x = np.asarray(x, dtype=np.complex128)
    V = np.asarray(V, dtype=np.complex128)
    frame = np.asarray(frame)
    k = np.asarray(k, dtype=np.float64)
    y = np.zeros((len(coil_idx), k.shape[0]), dtype=np.complex128)
    for t in np.unique(frame):
        sel = np.nonzero(frame == t)[0]
        Xt = np.tensordot(V[t], x, axes=(0, 0))
        for b, c in enumerate(coil_idx):
            y[b, sel] = nudft.type2(np.asarray(smaps[c]) * Xt, k[sel])
    return y
