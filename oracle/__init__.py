"""CPU FP64 oracle for iterative Grover search on matrix product states.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package. The
GPU library never calls it, and it shares no code with the HIP path: the only
common module is ``paper_2601_03832_amd.inputs``, which draws seeded inputs and
holds none of the method's arithmetic.

Contents (each function cites the passage of the paper it follows):

* :mod:`oracle.closed_form`  -- theta, P(k) and every amplitude of G^k|s> (Eqs. (2), (5), (6)).
* :mod:`oracle.statevector`  -- the plain definition: psi <- D O psi on 2^n amplitudes
  (Eqs. (3)-(4)); the gate-level circuit of Fig. 1(A); the dense 2^n x 2^n unitary.
* :mod:`oracle.mps`          -- the MPS method step by step (Section III-B): bond-2 MPO per
  reflection, QR left-canonicalisation sweep, truncated-SVD sweep, renormalisation,
  amplitudes, marked probability and perfect sampling. numpy LAPACK routines serve as steps.
* :mod:`oracle.philox`       -- Philox4x64-10 (Salmon et al., SC'11), the sampling RNG.
* :mod:`oracle.sampling`     -- exact site-by-site sampling from closed-form marginals.
"""
