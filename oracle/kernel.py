"""Kaiser-Bessel gridding kernel in FP64.  Test infrastructure only.

The paper names the NUFFT but fixes neither its kernel nor its accuracy
(Sec. 2.2, Sec. 3).  The reading taken here: a Kaiser-Bessel kernel of
width W (in fine-grid cells) on a grid oversampled by sigma, with the
width parameter of Beatty, Nishimura and Pauly (2005):

    beta = pi * sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8)

    phi(u) = I0(beta sqrt(1 - (2u/W)^2))     for |u| <= W/2, else 0

Its continuous Fourier transform (the deapodisation) in closed form is

    phi_hat(xi) = W sinh(sqrt(beta^2 - (pi W xi)^2)) / sqrt(beta^2 - (pi W xi)^2)

which stays real and positive for |xi| <= 1/(2 sigma) whenever
pi W / (2 sigma) < beta (true for W = 6, sigma = 2).
"""

import numpy as np
import scipy.special


def beta(W, sigma):
    """Kaiser-Bessel shape parameter for width W and oversampling sigma."""
    return np.pi * np.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def phi(u, W, b):
    """Kernel value at offset u (cells) from the point; zero outside."""
    u = np.asarray(u, dtype=np.float64)
    arg = 1.0 - (2.0 * u / W) ** 2
    inside = arg >= 0.0
    out = np.zeros_like(u)
    out[inside] = scipy.special.i0(b * np.sqrt(arg[inside]))
    return out


def phi_hat(xi, W, b):
    """Continuous Fourier transform of phi at frequency xi (cycles/cell)."""
    xi = np.asarray(xi, dtype=np.float64)
    z2 = b * b - (np.pi * W * xi) ** 2
    if np.any(z2 <= 0.0):
        raise ValueError("frequency outside the range where phi_hat is sinh-form")
    z = np.sqrt(z2)
    return W * np.sinh(z) / z


def _smooth(n):
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


def fine_size(n, sigma, W):
    """Smallest even 2,3,5,7-smooth length >= max(sigma*n, 2W)."""
    m = int(np.ceil(sigma * n - 1e-9))
    m = max(m, 2 * W)
    m += m % 2
    while not _smooth(m):
        m += 2
    return m
