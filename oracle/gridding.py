"""Oversampled gridding NUFFT in FP64, step by step.  Test infrastructure only.

The forward operator A of Sec. 2 contains a NUFFT.  This module evaluates it
the way a gridding NUFFT does, in the order of its definition and with no
blocking or fusion, so that each stage can be compared on its own:

type 2 (image -> k-space)
    1. deapodise and zero-pad: g[n mod nf] = f[n] / (phi_hat_z phi_hat_y phi_hat_x)
       with phi_hat_d = phi_hat(n_d / nf_d)
    2. unnormalised forward FFT (sign -) of the fine grid
    3. fine coordinate s = k nf / (2 pi); nodes l with s - W/2 < l <= s + W/2
       (half-open, exactly W nodes per axis: l = l0 .. l0+W-1 with
       l0 = floor(s - W/2) + 1)
    4. c_j = sum_l G[l mod nf] phi(s_x-l_x) phi(s_y-l_y) phi(s_z-l_z)

type 1 (k-space -> image) is the exact adjoint of the above:
    1. spread H[l mod nf] += c_j phi phi phi over the same W^3 nodes
    2. unnormalised inverse FFT (sign +), i.e. nf^3 * ifftn
    3. crop to the modes and deapodise

Why it works: by Poisson summation, sum_l phi(s-l) e^{-2 pi i n l / nf}
equals phi_hat(n/nf) e^{-i k n} plus aliased images that decay with the
kernel's spectrum, so deapodising by phi_hat recovers the exact NUDFT up to
that aliasing error.
"""

import os

import numpy as np
import scipy.fft

from . import kernel
from .nudft import modes

# FFT threads: the cores this process may use, capped by OMP_NUM_THREADS
_WORKERS = max(1, min(len(os.sched_getaffinity(0)),
                      int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or 1 << 30))


class Grid:
    """Fine-grid geometry and kernel parameters for an image shape."""

    def __init__(self, shape, sigma=2.0, W=6):
        self.shape = tuple(int(s) for s in shape)          # (Nz, Ny, Nx)
        self.sigma = float(sigma)
        self.W = int(W)
        self.beta = kernel.beta(self.W, self.sigma)
        self.nf = tuple(kernel.fine_size(n, self.sigma, self.W) for n in self.shape)
        # per axis: fine index of every mode, and the deapodisation factor
        self.pos = [modes(n) % nf for n, nf in zip(self.shape, self.nf)]
        self.dea = [kernel.phi_hat(modes(n) / nf, self.W, self.beta)
                    for n, nf in zip(self.shape, self.nf)]

    # -- per-axis kernel nodes and weights -----------------------------------
    def nodes(self, k):
        """Node start l0 [M,3] (x,y,z columns) and weights [M,3,W] for points k."""
        k = np.asarray(k, dtype=np.float64)
        nf_xyz = np.array(self.nf[::-1], dtype=np.float64)   # (nfx, nfy, nfz)
        s = k * nf_xyz / (2.0 * np.pi)
        l0 = np.floor(s - self.W / 2.0).astype(np.int64) + 1
        off = np.arange(self.W)
        u = s[:, :, None] - (l0[:, :, None] + off[None, None, :])
        w = kernel.phi(u, self.W, self.beta)
        return l0, w

    def _flat_nodes(self, l0, w):
        """Flat fine-grid indices [m, W^3] and weights [m, W^3]."""
        nfz, nfy, nfx = self.nf
        off = np.arange(self.W)
        lx = (l0[:, 0, None] + off) % nfx
        ly = (l0[:, 1, None] + off) % nfy
        lz = (l0[:, 2, None] + off) % nfz
        flat = ((lz[:, :, None, None] * nfy + ly[:, None, :, None]) * nfx
                + lx[:, None, None, :])
        ww = w[:, 2, :, None, None] * w[:, 1, None, :, None] * w[:, 0, None, None, :]
        m = l0.shape[0]
        return flat.reshape(m, -1), ww.reshape(m, -1)

    # -- type 2 stages ---------------------------------------------------------
    def deapodise_pad(self, f):
        f = np.asarray(f, dtype=np.complex128)
        if f.shape != self.shape:
            raise ValueError("image shape mismatch")
        g = np.zeros(self.nf, dtype=np.complex128)
        d = (self.dea[0][:, None, None] * self.dea[1][None, :, None]
             * self.dea[2][None, None, :])
        g[np.ix_(*self.pos)] = f / d
        return g

    @staticmethod
    def fft(g):
        return scipy.fft.fftn(g, workers=_WORKERS)

    def interp(self, G, k, chunk=65536):
        k = np.asarray(k, dtype=np.float64)
        m = k.shape[0]
        out = np.empty(m, dtype=np.complex128)
        Gf = G.ravel()
        for a in range(0, m, chunk):
            b = min(m, a + chunk)
            l0, w = self.nodes(k[a:b])
            flat, ww = self._flat_nodes(l0, w)
            out[a:b] = np.sum(Gf[flat] * ww, axis=1)
        return out

    def type2(self, f, k):
        return self.interp(self.fft(self.deapodise_pad(f)), k)

    # -- type 1 stages ---------------------------------------------------------
    def spread(self, c, k, chunk=65536):
        c = np.asarray(c, dtype=np.complex128).ravel()
        k = np.asarray(k, dtype=np.float64)
        size = int(np.prod(self.nf))
        re = np.zeros(size)
        im = np.zeros(size)
        for a in range(0, k.shape[0], chunk):
            b = min(k.shape[0], a + chunk)
            l0, w = self.nodes(k[a:b])
            flat, ww = self._flat_nodes(l0, w)
            v = ww * c[a:b, None]
            re += np.bincount(flat.ravel(), weights=v.real.ravel(), minlength=size)
            im += np.bincount(flat.ravel(), weights=v.imag.ravel(), minlength=size)
        return (re + 1j * im).reshape(self.nf)

    def ifft(self, H):
        return scipy.fft.ifftn(H, workers=_WORKERS) * float(np.prod(self.nf))

    def crop_deapodise(self, Hh):
        d = (self.dea[0][:, None, None] * self.dea[1][None, :, None]
             * self.dea[2][None, None, :])
        return Hh[np.ix_(*self.pos)] / d

    def type1(self, c, k):
        return self.crop_deapodise(self.ifft(self.spread(c, k)))


def type2(f, k, sigma=2.0, W=6):
    return Grid(np.shape(f), sigma, W).type2(f, k)


def type1(c, k, shape, sigma=2.0, W=6):
    return Grid(shape, sigma, W).type1(c, k)
