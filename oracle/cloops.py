"""Full-size gridding sums for the FP64 oracle.  Test infrastructure only.

``interp_many`` and ``spread_many`` compute what ``Grid.interp`` and
``Grid.spread`` compute (the sums over the W^3 kernel nodes of every point),
for several fine grids at once, with the triple sum in plain C loops
(``gridding_loops.c``, OpenMP over points or z planes).  The node indices
and weights still come from ``Grid.nodes``, so the kernel, the support rule
and the fine coordinate are the pinned NumPy ones; the tests pin these two
functions to ``Grid.interp`` / ``Grid.spread`` on small cases.

The C file is compiled with the system C compiler into ``oracle/_build/``
on first use (or by ``build()``).
"""

import ctypes
import os
import shutil
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gridding_loops.c")
_LIB = os.path.join(_HERE, "_build", "libgridding_loops.so")
_lib = None


def build(force=False):
    """Compile the C loops into oracle/_build/ (when missing or stale)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    cc = os.environ.get("CC") or shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler for the oracle's gridding loops")
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.run([cc, "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        i64, dp, lp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        for name in ("oracle_interp", "oracle_spread"):
            fn = getattr(L, name)
            fn.argtypes = [dp, i64, i64, i64, i64, i64, lp, dp, i64, dp]
            fn.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _nodes(grid, k):
    l0, w = grid.nodes(k)
    return (np.ascontiguousarray(l0, dtype=np.int64),
            np.ascontiguousarray(w, dtype=np.float64))


def node_chunks(grid, k, chunk=1 << 20):
    """Grid.nodes of the points k in chunks: [(start, stop, l0, w)], for
    reuse by several interp_many / spread_many calls on the same points."""
    k = np.asarray(k, dtype=np.float64)
    return [(a, min(k.shape[0], a + chunk)) + _nodes(grid, k[a:min(k.shape[0], a + chunk)])
            for a in range(0, k.shape[0], chunk)]


def interp_many(grid, Gs, k, chunk=1 << 20, nodes=None):
    """out[p, j] = Grid.interp(Gs[p], k)[j] for fine grids Gs [P, nfz, nfy, nfx]
    (``nodes``: node_chunks of the same points, else computed here)."""
    L = _load()
    Gs = np.ascontiguousarray(Gs, dtype=np.complex128)
    if Gs.ndim == 3:
        Gs = Gs[None]
    P = Gs.shape[0]
    nfz, nfy, nfx = grid.nf
    if Gs.shape[1:] != (nfz, nfy, nfx):
        raise ValueError("grid shape mismatch")
    k = np.asarray(k, dtype=np.float64)
    m = k.shape[0]
    out = np.empty((P, m), dtype=np.complex128)
    for a, b, l0, w in (nodes if nodes is not None else node_chunks(grid, k, chunk)):
        part = np.empty((P, b - a), dtype=np.complex128)
        L.oracle_interp(_dp(Gs.view(np.float64)), P, nfz, nfy, nfx, grid.W,
                        l0.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(w), b - a,
                        _dp(part.view(np.float64)))
        out[:, a:b] = part
    return out


def spread_many(grid, cs, k, chunk=1 << 20, nodes=None):
    """H[p] = Grid.spread(cs[p], k) for values cs [P, M] (``nodes`` as for
    interp_many)."""
    L = _load()
    cs = np.ascontiguousarray(cs, dtype=np.complex128)
    if cs.ndim == 1:
        cs = cs[None]
    P = cs.shape[0]
    nfz, nfy, nfx = grid.nf
    k = np.asarray(k, dtype=np.float64)
    m = k.shape[0]
    H = np.zeros((P, nfz, nfy, nfx), dtype=np.complex128)
    for a, b, l0, w in (nodes if nodes is not None else node_chunks(grid, k, chunk)):
        v = np.ascontiguousarray(cs[:, a:b])
        L.oracle_spread(_dp(v.view(np.float64)), P, nfz, nfy, nfx, grid.W,
                        l0.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(w), b - a,
                        _dp(H.view(np.float64)))
    return H
