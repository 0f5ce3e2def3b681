"""Dense truth and residual certificates (TEST INFRASTRUCTURE).

The problem statement (Sec. 1, eq. psvd): all singular triplets
(sigma_i, u_i, v_i) of a real m x n matrix A (m >= n) with sigma_i in the
closed interval [a, b], 0 <= a < b.  For sizes where a dense SVD fits, the
truth is LAPACK's SVD of A (numpy.linalg.svd, dgesdd).
"""
from __future__ import annotations

import numpy as np

from .method import as_dense


def dense_truth(A, a, b):
    """All singular triplets with a <= sigma <= b, ascending sigma."""
    Ad = as_dense(A)
    U, s, Vt = np.linalg.svd(Ad, full_matrices=False)
    sel = np.nonzero((s >= a) & (s <= b))[0]
    sel = sel[np.argsort(s[sel], kind="stable")]
    V = Vt.T[:, sel]
    Uu = U[:, sel]
    for i in range(len(sel)):
        j = int(np.argmax(np.abs(V[:, i])))
        if V[j, i] < 0:
            V[:, i] = -V[:, i]
            Uu[:, i] = -Uu[:, i]
    return s[sel], Uu, V, s


def norm2(A):
    """||A||_2 from the dense SVD."""
    return float(np.linalg.svd(as_dense(A), compute_uv=False)[0])


def triplet_residuals(A, sigma, U, V, normA=None):
    """max(||A v - sigma u||, ||A^T u - sigma v||) / ||A||_2 per triplet, i.e.
    the residual 2-norm used in the experiments (Sec. 4.2) made relative to
    the matrix norm as in the normalised setting of Sec. 4.3."""
    Ad = as_dense(A)
    if normA is None:
        normA = norm2(Ad)
    r1 = np.linalg.norm(Ad @ V - U * sigma[None, :], axis=0)
    r2 = np.linalg.norm(Ad.T @ U - V * sigma[None, :], axis=0)
    return np.maximum(r1, r2) / normA


def sparse_triplet_residuals(rowptr, colidx, vals, m, n, sigma, U, V, normA):
    """The residuals of ``triplet_residuals`` where no dense copy of A fits:
    A V and A^T U are taken with a CSR library product (scipy.sparse)."""
    import scipy.sparse as sp
    A = sp.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(colidx), np.asarray(rowptr)), shape=(m, n))
    r1 = np.linalg.norm(A @ V - U * sigma[None, :], axis=0)
    r2 = np.linalg.norm(A.T @ U - V * sigma[None, :], axis=0)
    return np.maximum(r1, r2) / normA


def sparse_norm2_lower(rowptr, colidx, vals, m, n, iters=100, seed=0):
    """A lower bound of ||A||_2 from the power method on A^T A (seeded start):
    the Rayleigh quotient x^T A^T A x / x^T x never exceeds ||A||_2^2, so a
    residual divided by this bound is not understated."""
    import scipy.sparse as sp
    A = sp.csr_matrix((np.asarray(vals, dtype=np.float64), np.asarray(colidx), np.asarray(rowptr)), shape=(m, n))
    x = np.random.default_rng(seed).standard_normal(n)
    lam = 0.0
    for _ in range(iters):
        x /= np.linalg.norm(x)
        y = A.T @ (A @ x)
        lam = max(lam, float(x @ y))
        x = y
    return float(np.sqrt(lam))


def strict_count(s, a, b, band):
    """Number of sigma strictly inside (a + band, b - band) and the number in
    the edge bands [a - band, a + band] and [b - band, b + band]."""
    s = np.asarray(s)
    strict = int(np.sum((s > a + band) & (s < b - band)))
    edge = int(np.sum((np.abs(s - a) <= band) | (np.abs(s - b) <= band)))
    return strict, edge


def subspace_gap(X, Y):
    """sin of the largest principal angle between span(X) and span(Y), both
    given by orthonormal columns of the same count: the 2-norm of the part
    of Y outside span(X), (I - X X^T) Y.  Taking the sine directly (not
    sqrt(1 - cos^2)) keeps small angles accurate."""
    if X.shape[1] == 0 and Y.shape[1] == 0:
        return 0.0
    if X.shape[1] != Y.shape[1]:
        raise ValueError("subspaces of different dimension")
    D = Y - X @ (X.T @ Y)
    return float(np.linalg.norm(D, 2))
