"""CPU FP64 oracle for the multicoil subspace NUFFT of StoDIP (arXiv 2408.02367).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library; the two meet only on the seeded inputs of
``workloads``.

What it computes (Sec. 2, Eq. 1-3 of the paper):

* ``nudft``    - the plain definitions of the type-2 (uniform -> nonuniform)
                 and type-1 (nonuniform -> uniform) nonuniform DFTs.  This is
                 the truth every other result is judged against.
* ``kernel``   - the Kaiser-Bessel gridding kernel, its width parameter and
                 its continuous Fourier transform (deapodisation).
* ``gridding`` - the oversampled gridding NUFFT (deapodise, zero-pad, FFT,
                 interpolate; and the exact adjoint: spread, IFFT, crop,
                 deapodise), step by step in FP64.
* ``cloops``   - the same node sums as ``gridding``'s interpolation and
                 spreading, as plain C loops over several grids at once
                 (``gridding_loops.c``), for full-size comparisons.
* ``mrf``      - the MRF forward operator A_c (coil sensitivities, NUFFT,
                 temporal-subspace mix), its adjoint, the data-consistency
                 loss of Eq. 2-3 and its gradient 2 A^H w (A x - d), plus a
                 frame-expansion brute force for tiny sizes.
* ``dcf``      - the density compensation weights of Eq. 2 by Pipe-Menon
                 fixed-point iteration with the gridding kernel.
* ``tv``       - the total-variation penalty of Alg. 1 (StoDIP + TV) and its
                 gradient.
* ``recon``    - the initialisers of Sec. 2.2: normal operator over all
                 coils, conjugate gradients (with and without Tikhonov) and
                 the scaled adjoint.

Every function is pinned by the ``-m "not gpu"`` tests in ``tests/`` to
something other than itself (library FFTs on on-grid points, closed forms,
Parseval, adjoint identities, quadrature, brute-force loops).
"""

from . import nudft, kernel, gridding, cloops, mrf, dcf, tv, recon  # noqa: F401
