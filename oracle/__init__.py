"""CPU FP64 oracle for the complex moment-based interior SVD (TEST INFRASTRUCTURE).

This package is test infrastructure only.  It is a plain, slow, obviously
correct NumPy implementation of what the GPU path computes, written from the
paper (Imakura & Sakurai, "Complex moment-based method with nonlinear
transformation for computing large and sparse interior singular triplets").
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library and never
imports it; the only thing both sides share is the seeded input generator
module ``synth``.

Modules
-------
quadrature  ellipse trapezoid rule, nonlinear transform, filter functions
            (Sec. 4 quadrature definition; Sec. 3.2 filter f; Sec. 3.3 f_g).
method      Algorithms 1 and 2 step by step with dense direct shifted solves,
            spurious index and practical residual estimates (Sec. 3.4).
truth       dense LAPACK SVD truth and triplet residual certificates.
krylov      a plain per-shift COCG solver for sizes where dense solves do not
            fit (used for CPU timing samples and moderate-size checks).
sparse      CSR transpose and row-sampled products by their definitions.

Parity status: every function is pinned by tests in ``tests/test_oracle_pins.py``
against closed forms, invariants or exact spectra; none is "parity unpinned".
"""
from . import quadrature, method, truth, krylov, sparse  # noqa: F401
