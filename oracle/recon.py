"""Initialisers of the TSMI x^(0), FP64.

Test infrastructure only.

Sec. 2.2 starts the network from an estimate of the inverse problem of
Eq. 1 rather than from noise, by (a) the SVD-MRF adjoint with a scaling
factor, (b) low-rank least squares by conjugate gradients and (c) the same
with Tikhonov regularisation.  The paper names the three and no more; the
readings taken here, over all C coils with the DCF weight W = diag(w):

    normal operator   N(x) = sum_c A_c^H W A_c x + lam x
                      (lam = 0 for (b), lam > 0 for (c); "low rank" is the
                      K-channel subspace of the TSMI)
    right-hand side   b = sum_c A_c^H W y_c
    CG                the textbook conjugate-gradient iteration on
                      N x = b from x0, a fixed number of iterations
    scaled adjoint    z = b and the s that minimises
                      sum_c || W^1/2 (y_c - s A_c z) ||^2, which is
                      s = <z, z> / sum_c <A_c z, W A_c z>  (real, since
                      Re <A_c z, W y_c> summed over c is <z, b> = |z|^2)

Every operator is ``oracle.mrf``'s forward/adjoint with coils 0..C-1.
"""

import numpy as np

from . import mrf


def _w(w, M):
    return np.ones(M) if w is None else np.asarray(w, dtype=np.float64)


def normal(op, x, smaps, V, frame, k, w=None, lam=0.0):
    """sum_c A_c^H W A_c x + lam x."""
    C = np.shape(smaps)[0]
    coils = list(range(C))
    y = mrf.forward(op, x, smaps, coils, V, frame, k)
    y = y * _w(w, y.shape[1])[None, :]
    return mrf.adjoint(op, y, smaps, coils, V, frame, k, np.shape(x)[0]) + lam * np.asarray(x)


def rhs(op, y, smaps, V, frame, k, K, w=None):
    """sum_c A_c^H W y_c for y[C, M]."""
    y = np.asarray(y, dtype=np.complex128)
    C = np.shape(smaps)[0]
    return mrf.adjoint(op, y * _w(w, y.shape[1])[None, :], smaps, list(range(C)), V, frame, k, K)


def _dot(a, b):
    return complex(np.vdot(a, b))


def cg(op, y, smaps, V, frame, k, x0, iterations, w=None, lam=0.0):
    """x after ``iterations`` CG steps on N x = b, and |r|^2 before each step
    and after the last (iterations + 1 values)."""
    x = np.array(x0, dtype=np.complex128)
    b = rhs(op, y, smaps, V, frame, k, x.shape[0], w)
    r = b - normal(op, x, smaps, V, frame, k, w, lam)
    p = r.copy()
    rs = _dot(r, r).real
    hist = [rs]
    for _ in range(int(iterations)):
        Ap = normal(op, p, smaps, V, frame, k, w, lam)
        alpha = rs / _dot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        rs_new = _dot(r, r).real
        p = r + (rs_new / rs) * p
        rs = rs_new
        hist.append(rs)
    return x, np.array(hist)


def scaled_adjoint(op, y, smaps, V, frame, k, K, w=None):
    """(s z, s) with z = b and s the least-squares scale."""
    z = rhs(op, y, smaps, V, frame, k, K, w)
    C = np.shape(smaps)[0]
    Az = mrf.forward(op, z, smaps, list(range(C)), V, frame, k)
    den = float(np.sum(_w(w, Az.shape[1])[None, :] * np.abs(Az) ** 2))
    s = _dot(z, z).real / den
    return s * z, s
