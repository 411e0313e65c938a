"""Density compensation by Pipe-Menon fixed-point iteration, FP64.
Test infrastructure only.

The loss of Eq. 2 weights every k-space sample by a density compensation
function (DCF, Sec. 2). The paper does not say how it computes the DCF;
the reading taken here is the Pipe-Menon iteration (Pipe & Menon, MRM 1999)
with the gridding kernel of the NUFFT, normalised to 1 at its centre on
every axis:

    w_0 = 1,    w_{n+1} = w_n / (C w_n),
    (C w)_j = sum_l phi~(s_j - l) sum_i phi~(s_i - l) w_i,

i.e. spreading w onto the fine grid and interpolating back (no FFT, no
deapodisation), with phi~ = phi / I0(beta) per axis and the half-open node
rule of the gridding NUFFT.
"""

import numpy as np

from . import kernel


def convolve(grid, k, w):
    """(C w)_j for points k [M, 3] and real weights w [M] (normalised kernel)."""
    peak = float(kernel.phi(0.0, grid.W, grid.beta))
    H = grid.spread(np.asarray(w, dtype=np.float64).astype(np.complex128), k)
    return grid.interp(H, k).real / peak ** 6


def pipe_menon(grid, k, iterations):
    """DCF after ``iterations`` Pipe-Menon updates, starting from w = 1."""
    w = np.ones(np.asarray(k).shape[0])
    for _ in range(int(iterations)):
        w = w / convolve(grid, k, w)
    return w
