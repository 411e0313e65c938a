"""Seeded synthetic inputs shaped like whole-brain 3D MRF (Sec. 3.1).

The paper's in-vivo scans are private, so these generators stand in for
them with the same structure: 3D spiral-projection trajectories whose every
arm crosses the k-space centre, a smooth piecewise-constant multi-tissue
subspace image, smooth coil-sensitivity maps normalised to unit
root-sum-of-squares, and a random orthonormal temporal basis.

This module holds none of the operator's arithmetic: it only draws inputs.
Both the HIP path and the CPU oracle consume what it returns.  Every draw
uses ``numpy.random.default_rng([seed, component])`` so that each component
can be regenerated on its own.
"""

import numpy as np

# component ids for the seeded generators
IMAGE, TRAJ, COILS, BASIS, NOISE, PERTURB, COIL_DRAW, KSPACE = range(8)

# 2D golden means used for the 3D rotation of spiral arms
_PHI1, _PHI2 = 0.4656, 0.6823
KMAX = np.pi * (1.0 - 2.0 ** -20)


def rng(seed, component):
    return np.random.default_rng([int(seed), int(component)])


def spiral_trajectory(T, L, S, turns=None, kmax=KMAX):
    """3D spiral-projection trajectory: T frames x L interleaves x S samples.

    Each arm a = t*L + l is a planar Archimedean spiral from the k-space
    centre to radius ``kmax`` (radians per voxel) with ``turns`` turns
    (default S/64), rotated by a golden-means 3D rotation.  Points are
    ordered (t, l, s), t slowest.  Returns (traj float32 [M, 3] with
    columns (kx, ky, kz), frame_of_point int32 [M]).
    """
    if turns is None:
        turns = S / 64.0
    a = np.arange(T * L, dtype=np.float64)
    s = np.arange(S, dtype=np.float64) / max(S - 1, 1)
    r = kmax * s
    th = 2.0 * np.pi * turns * s
    local = np.stack([r * np.cos(th), r * np.sin(th), np.zeros_like(r)], axis=1)
    g1 = np.mod(a * _PHI1, 1.0)
    g2 = np.mod(a * _PHI2, 1.0)
    az = 2.0 * np.pi * g2
    pol = np.arccos(1.0 - 2.0 * g1)
    tw = a * np.pi * (3.0 - np.sqrt(5.0))

    def rz(t):
        c, s_ = np.cos(t), np.sin(t)
        R = np.zeros((t.size, 3, 3))
        R[:, 0, 0], R[:, 0, 1], R[:, 1, 0], R[:, 1, 1], R[:, 2, 2] = c, -s_, s_, c, 1.0
        return R

    def ry(t):
        c, s_ = np.cos(t), np.sin(t)
        R = np.zeros((t.size, 3, 3))
        R[:, 0, 0], R[:, 0, 2], R[:, 2, 0], R[:, 2, 2], R[:, 1, 1] = c, s_, -s_, c, 1.0
        return R

    R = rz(az) @ ry(pol) @ rz(tw)                       # [A, 3, 3]
    traj = np.einsum("aij,sj->asi", R, local).reshape(-1, 3)
    traj = np.clip(traj, -kmax, kmax).astype(np.float32)
    frame = np.repeat(np.arange(T, dtype=np.int32), L * S)
    return traj, frame


def random_image(shape, seed, batch=None):
    """i.i.d. N(0,1) real and imaginary parts, complex64."""
    g = rng(seed, IMAGE)
    sh = tuple(shape) if batch is None else (batch,) + tuple(shape)
    return (g.standard_normal(sh) + 1j * g.standard_normal(sh)).astype(np.complex64)


def _axis_coords(n):
    return (np.arange(n, dtype=np.float64) - n // 2) / n   # FOV [-1/2, 1/2)


def phantom(shape, K, seed, blur=1.0):
    """Smooth piecewise-constant tissue phantom x[K, Nz, Ny, Nx] (complex64).

    A head ellipsoid plus 2-4 inner ellipsoids (3-5 tissue classes in all),
    each class with its own complex N(0,1) K-vector, background zero, then a
    Gaussian blur of ``blur`` voxels.
    """
    import scipy.ndimage

    g = rng(seed, IMAGE)
    nz, ny, nx = shape
    z = _axis_coords(nz)[:, None, None]
    y = _axis_coords(ny)[None, :, None]
    x = _axis_coords(nx)[None, None, :]
    ncls = int(g.integers(3, 6))
    label = np.full(shape, -1, dtype=np.int8)
    head = (x / 0.40) ** 2 + (y / 0.44) ** 2 + (z / 0.38) ** 2 <= 1.0
    label[head] = 0
    for c in range(1, ncls):
        ctr = g.uniform(-0.15, 0.15, 3)
        ax = g.uniform(0.10, 0.35, 3) * 0.6
        inside = (((x - ctr[0]) / ax[0]) ** 2 + ((y - ctr[1]) / ax[1]) ** 2
                  + ((z - ctr[2]) / ax[2]) ** 2 <= 1.0) & head
        label[inside] = c
    vec = g.standard_normal((ncls, K)) + 1j * g.standard_normal((ncls, K))
    out = np.zeros((K,) + tuple(shape), dtype=np.complex64)
    for k in range(K):
        vol = np.zeros(shape, dtype=np.complex64)
        for c in range(ncls):
            vol[label == c] = vec[c, k]
        if blur:
            vol = (scipy.ndimage.gaussian_filter(vol.real, blur)
                   + 1j * scipy.ndimage.gaussian_filter(vol.imag, blur))
        out[k] = vol
    return out


def coil_maps(shape, C, seed, radius=0.6, width=0.35, max_cycles=1.0, select=None):
    """C smooth coil maps S[C, Nz, Ny, Nx] (complex64) with sqrt(sum |S_c|^2) = 1.

    Gaussian-bump magnitudes centred on a Fibonacci sphere of ``radius``
    (FOV units) and a random linear phase of at most ``max_cycles`` cycles
    per FOV.  Both factors are separable over the axes.  ``select`` (indices)
    returns only those maps, normalised by the root-sum-of-squares of all C.
    """
    g = rng(seed, COILS)
    nz, ny, nx = shape
    ax = [_axis_coords(nx), _axis_coords(ny), _axis_coords(nz)]
    i = np.arange(C) + 0.5
    polar = np.arccos(1.0 - 2.0 * i / C)
    azim = np.pi * (1.0 + 5.0 ** 0.5) * i
    ctr = radius * np.stack([np.sin(polar) * np.cos(azim),
                             np.sin(polar) * np.sin(azim), np.cos(polar)], axis=1)
    gdir = g.standard_normal((C, 3))
    gdir /= np.linalg.norm(gdir, axis=1, keepdims=True)
    gvec = gdir * g.uniform(0.0, max_cycles, (C, 1))
    keep = list(range(C)) if select is None else [int(c) for c in select]
    maps = np.empty((len(keep),) + tuple(shape), dtype=np.complex64)
    rss = np.zeros(shape, dtype=np.float64)
    for c in range(C):
        f = [np.exp(-(ax[d] - ctr[c, d]) ** 2 / (2 * width ** 2))
             * np.exp(2j * np.pi * gvec[c, d] * ax[d]) for d in range(3)]
        m = f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]
        if c in keep:
            maps[keep.index(c)] = m
        rss += np.abs(m) ** 2
    maps /= np.sqrt(rss).astype(np.float32)[None]
    return maps


def subspace_basis(T, K, seed):
    """Random orthonormal temporal basis V[T, K] (complex64): Q of a QR."""
    g = rng(seed, BASIS)
    a = g.standard_normal((T, K)) + 1j * g.standard_normal((T, K))
    q, _ = np.linalg.qr(a)
    return q.astype(np.complex64)


def coil_minibatch(C, B, seed, step=0):
    """Coil indices of minibatch ``step``: consecutive chunks of a seeded
    random permutation of the C coils (drawn without replacement)."""
    per_epoch = C // B
    epoch, part = divmod(step, per_epoch)
    perm = rng(seed * 1000003 + epoch, COIL_DRAW).permutation(C)
    return perm[part * B:(part + 1) * B].astype(np.int32)


def complex_noise(shape, rel, ref_rms, seed):
    """Complex Gaussian noise of std rel * ref_rms (split over re and im)."""
    g = rng(seed, NOISE)
    s = rel * np.asarray(ref_rms, dtype=np.float64) / np.sqrt(2.0)
    if np.ndim(s):
        s = s.reshape(s.shape + (1,) * (len(shape) - s.ndim))
    return (s * (g.standard_normal(shape) + 1j * g.standard_normal(shape))).astype(np.complex64)


def random_kspace(shape, seed):
    g = rng(seed, KSPACE)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)


# ---------------------------------------------------------------------------
# The workloads.  Each entry is a geometry; arrays are drawn on demand.
# ---------------------------------------------------------------------------
CONFIGS = {
    # plain 3D NUFFT: 32^3 image, 64^3 grid, 8 arms x 1024 samples
    "c1": dict(shape=(32, 32, 32), K=1, C=1, B=1, T=1, L=8, S=1024),
    # MRF subspace geometry at 160^3, K=5, 32 coils, M = 9.6M
    "c2": dict(shape=(160, 160, 160), K=5, C=32, B=1, T=1000, L=8, S=1200),
    # batched: 4-of-32 coils x K=5 on the c2 geometry
    "c3": dict(shape=(160, 160, 160), K=5, C=32, B=4, T=1000, L=8, S=1200),
    # ragged volumes (same sample density as c2, T proportional to voxels)
    "c3r128": dict(shape=(128, 128, 128), K=5, C=32, B=4, T=512, L=8, S=1200),
    "c3r192": dict(shape=(160, 192, 192), K=5, C=32, B=4, T=1440, L=8, S=1200),
    # differentiable DC step on the c3 geometry
    "c4": dict(shape=(160, 160, 160), K=5, C=32, B=4, T=1000, L=8, S=1200),
    # large DC step: 224^3 x K=6, 8-of-48 coils, M = 20.16M
    "c5": dict(shape=(224, 224, 224), K=6, C=48, B=8, T=1200, L=12, S=1400),
    # the paper's own iteration shape (Sec. 3: 200^3 volume, 8 coils, 880
    # frames, 28 spiral arms per frame at R = 2, 876 samples per arm; one
    # coil per stochastic step as in Alg. 1), K = 5 channels: M = 21.59M
    "paper": dict(shape=(200, 200, 200), K=5, C=8, B=1, T=880, L=28, S=876),
    # the batched step at the plain-NUFFT geometry (32^3, 64^3 grid, 8192
    # points): the launch-latency-bound case
    "small": dict(shape=(32, 32, 32), K=5, C=8, B=4, T=8, L=1, S=1024),
}
SEEDS = {"c1": 1, "c2": 2, "c3": 3, "c3r128": 31, "c3r192": 32, "c4": 4, "c5": 5, "paper": 6,
         "small": 7}


def make(name, with_images=True, minibatch_maps=False):
    """Draw the inputs of workload ``name`` as numpy arrays.

    ``minibatch_maps``: keep only the coil maps of the minibatch (in
    minibatch order, still normalised over all C coils); ``coil_idx`` is
    then 0 .. B-1 and ``coil_idx_global`` the coils they stand for.
    """
    cfg = dict(CONFIGS[name])
    seed = SEEDS[name]
    traj, frame = spiral_trajectory(cfg["T"], cfg["L"], cfg["S"])
    out = dict(cfg, name=name, seed=seed, traj=traj, frame=frame)
    if with_images:
        if name == "c1":
            out["x"] = random_image(cfg["shape"], seed, batch=1)
            out["smaps"] = None
            out["V"] = None
        else:
            out["x"] = phantom(cfg["shape"], cfg["K"], seed)
            out["V"] = subspace_basis(cfg["T"], cfg["K"], seed)
        ci = coil_minibatch(cfg["C"], cfg["B"], seed)
        out["coil_idx"] = ci
        if name != "c1":
            if minibatch_maps:
                out["smaps"] = coil_maps(cfg["shape"], cfg["C"], seed, select=ci)
                out["coil_idx_global"] = ci
                out["coil_idx"] = np.arange(len(ci), dtype=np.int32)
            else:
                out["smaps"] = coil_maps(cfg["shape"], cfg["C"], seed)
    return out
