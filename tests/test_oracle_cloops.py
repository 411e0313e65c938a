"""Pins of the oracle's C gridding loops (CPU only).

``oracle.cloops`` evaluates the same node sums as ``Grid.interp`` and
``Grid.spread`` (which ``test_oracle.py`` pins to the direct NUDFT, to
adjoint identities and to brute force), for several grids at once.  These
tests tie the two together on small grids with ragged sizes, coordinates at
the +-pi edges, several chunks and several thread counts, and pin the C
type 2 / type 1 directly against the direct NUDFT as well.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import cloops, gridding, nudft


def _case(seed, shape=(10, 12, 14), M=3000, P=3):
    g = gridding.Grid(shape)
    rng = np.random.default_rng(seed)
    k = rng.uniform(-np.pi, np.pi, (M, 3))
    k[:10] = np.pi * (1 - 1e-12)       # just below +pi: wraps to the far edge
    k[10:20] = -np.pi
    k[20:30] = 0.0
    Gs = rng.standard_normal((P,) + g.nf) + 1j * rng.standard_normal((P,) + g.nf)
    cs = rng.standard_normal((P, M)) + 1j * rng.standard_normal((P, M))
    return g, k, Gs, cs


def test_interp_many_equals_numpy_interp():
    g, k, Gs, _ = _case(1)
    out = cloops.interp_many(g, Gs, k, chunk=700)
    ref = np.stack([g.interp(G, k) for G in Gs])
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_spread_many_equals_numpy_spread():
    g, k, _, cs = _case(2)
    H = cloops.spread_many(g, cs, k, chunk=700)
    ref = np.stack([g.spread(c, k) for c in cs])
    assert np.max(np.abs(H - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_c_type2_type1_match_direct_nudft():
    shape = (9, 8, 11)
    g = gridding.Grid(shape)
    rng = np.random.default_rng(3)
    k = rng.uniform(-np.pi, np.pi, (2500, 3))
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    c2 = cloops.interp_many(g, g.fft(g.deapodise_pad(f)), k)[0]
    assert np.linalg.norm(c2 - nudft.type2(f, k)) / np.linalg.norm(c2) < 2e-5
    c = rng.standard_normal(2500) + 1j * rng.standard_normal(2500)
    f1 = g.crop_deapodise(g.ifft(cloops.spread_many(g, c, k)[0]))
    ref = nudft.type1(c, k, shape)
    assert np.linalg.norm(f1 - ref) / np.linalg.norm(ref) < 2e-5


def test_interp_and_spread_are_adjoint():
    g, k, Gs, cs = _case(4, P=2)
    u = cloops.interp_many(g, Gs, k)
    H = cloops.spread_many(g, cs, k)
    lhs = np.vdot(cs, u)
    rhs = np.vdot(H, Gs)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("threads", ["1", "3"])
def test_results_do_not_depend_on_thread_count(threads):
    """The spread adds a cell's terms in point order whatever the number of
    threads, so it is bit-identical; interpolation has no shared sums."""
    code = ("import sys, numpy as np; sys.path.insert(0, %r);"
            "from oracle import cloops, gridding;"
            "g = gridding.Grid((10, 12, 14)); r = np.random.default_rng(5);"
            "k = r.uniform(-np.pi, np.pi, (4000, 3));"
            "c = r.standard_normal((2, 4000)) + 1j * r.standard_normal((2, 4000));"
            "H = cloops.spread_many(g, c, k);"
            "u = cloops.interp_many(g, H, k);"
            "sys.stdout.buffer.write(H.tobytes() + u.tobytes())"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    cloops.build()
    outs = []
    for t in ("1", threads if threads != "1" else "2"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True).stdout)
    assert outs[0] == outs[1]
