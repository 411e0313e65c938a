"""Direct (exact) nonuniform DFTs in FP64.  Test infrastructure only.

Definitions (Sec. 2: the NUFFT inside the forward operator A):

* modes   n in I_N = prod_d {-floor(N_d/2), ..., ceil(N_d/2)-1}; an image
          array f[z, y, x] holds mode n at index i_d = n_d + floor(N_d/2);
* points  k_j = (kx, ky, kz) in radians per voxel; column 0 pairs with the
          x axis (last array axis), column 2 with z (first array axis);
* type 2  c_j = sum_n f[n] exp(-i k_j . n)          (image -> k-space)
* type 1  f[n] = sum_j c_j exp(+i k_j . n)          (k-space -> image)

Type 1 is the exact adjoint of type 2.  Both are evaluated by separable
contractions with E_d[j, n_d] = exp(-i k_{j,d} n_d), chunked over points;
coordinates are upcast exactly from whatever precision the caller holds.
"""

import numpy as np


def modes(n):
    """Mode numbers of one axis of length n, in array order."""
    return np.arange(n, dtype=np.int64) - n // 2


def _as_points(k):
    k = np.asarray(k)
    if k.ndim != 2 or k.shape[1] != 3:
        raise ValueError("points must be an [M, 3] array (kx, ky, kz)")
    return k.astype(np.float64)


def type2(f, k, chunk=1024):
    """c_j = sum_n f[n] exp(-i k_j.n) for an image f[Nz, Ny, Nx]."""
    f = np.asarray(f, dtype=np.complex128)
    nz, ny, nx = f.shape
    k = _as_points(k)
    m = k.shape[0]
    out = np.empty(m, dtype=np.complex128)
    mx, my, mz = modes(nx), modes(ny), modes(nz)
    f2 = f.reshape(nz * ny, nx)
    for a in range(0, m, chunk):
        b = min(m, a + chunk)
        ex = np.exp(-1j * np.outer(k[a:b, 0], mx))      # [m, Nx]
        ey = np.exp(-1j * np.outer(k[a:b, 1], my))      # [m, Ny]
        ez = np.exp(-1j * np.outer(k[a:b, 2], mz))      # [m, Nz]
        t1 = (f2 @ ex.T).reshape(nz, ny, b - a)          # sum over x
        t2 = np.einsum("zyj,jy->zj", t1, ey)             # sum over y
        out[a:b] = np.einsum("zj,jz->j", t2, ez)         # sum over z
    return out


def type1(c, k, shape, sel=None, chunk=4096):
    """f[n] = sum_j c_j exp(+i k_j.n) on an image of shape (Nz, Ny, Nx).

    ``sel`` optionally restricts the output to a Cartesian product of array
    indices ``(iz, iy, ix)``; the result then has shape
    ``(len(iz), len(iy), len(ix))``.
    """
    c = np.asarray(c, dtype=np.complex128).ravel()
    k = _as_points(k)
    nz, ny, nx = shape
    mz, my, mx = modes(nz), modes(ny), modes(nx)
    if sel is not None:
        iz, iy, ix = (np.asarray(s, dtype=np.int64) for s in sel)
        mz, my, mx = mz[iz], my[iy], mx[ix]
    out = np.zeros((len(mz) * len(my), len(mx)), dtype=np.complex128)
    m = k.shape[0]
    for a in range(0, m, chunk):
        b = min(m, a + chunk)
        ex = np.exp(1j * np.outer(k[a:b, 0], mx))
        ey = np.exp(1j * np.outer(k[a:b, 1], my))
        ez = np.exp(1j * np.outer(k[a:b, 2], mz))
        q = (c[a:b, None, None] * ez[:, :, None] * ey[:, None, :])
        out += q.reshape(b - a, -1).T @ ex
    return out.reshape(len(mz), len(my), len(mx))
