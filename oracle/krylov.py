"""Plain per-shift COCG for the shifted block systems (TEST INFRASTRUCTURE).

For sizes where the dense direct solves of ``method`` do not fit, the shifted
systems (z_j I - A^T A) Y_j = V (Algorithm 1, steps 1-2) are solved by the
conjugate orthogonal conjugate gradient method (COCG) for complex symmetric
matrices, one system per shift, all right-hand sides in lock step with their
own scalars.  The operator is applied as z P - A^T (A P) with two sparse
products; A^T A is never formed.  The bilinear form x^T y (no conjugation) is
the one COCG uses for complex symmetric matrices.
"""
from __future__ import annotations

import time

import numpy as np


def _csr(A):
    import scipy.sparse as sp
    if sp.issparse(A):
        return A.tocsr()
    if isinstance(A, np.ndarray):
        return sp.csr_matrix(A)
    return A.scipy()


def apply_shifted(Acsr, AT, z, P):
    """(z I - A^T A) P."""
    return z * P - AT @ (Acsr @ P)


def cocg(A, z, V, tol=1e-10, maxit=100000, time_limit=None):
    """Solve (z I - A^T A) Y = V column by column (columns in lock step).

    Stops when every column's residual ||V - (zI - A^T A) Y|| / ||V|| <= tol,
    after ``maxit`` iterations, or after ``time_limit`` seconds.  Returns
    (Y, iterations, relative residuals per column, seconds).
    """
    Acsr = _csr(A)
    AT = Acsr.T.tocsr()
    V = np.asarray(V, dtype=np.float64)
    Y = np.zeros(V.shape, dtype=np.complex128)
    R = V.astype(np.complex128)
    P = R.copy()
    rho = np.sum(R * R, axis=0)
    vn = np.linalg.norm(V, axis=0)
    vn[vn == 0] = 1.0
    t0 = time.perf_counter()
    it = 0
    res = np.linalg.norm(R, axis=0) / vn
    while it < maxit and res.max() > tol:
        Qv = apply_shifted(Acsr, AT, z, P)
        mu = np.sum(P * Qv, axis=0)
        alpha = rho / mu
        Y += alpha[None, :] * P
        R -= alpha[None, :] * Qv
        rho_new = np.sum(R * R, axis=0)
        beta = rho_new / rho
        rho = rho_new
        P = R + beta[None, :] * P
        it += 1
        res = np.linalg.norm(R, axis=0) / vn
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
    return Y, it, res, time.perf_counter() - t0
