"""Seeded synthetic inputs for the interior-SVD workloads.

This module only *builds inputs*: sparse matrices with known or random spectra,
right-hand-side blocks and target intervals.  It holds none of the method's
arithmetic (no quadrature, no shifted solves, no moments, no projections), so
both the CPU oracle and the GPU path consume the very same arrays.

Every generator draws from ``numpy.random.default_rng(SeedSequence([2109,
13655, config, instance]))`` so that a (config, instance) pair always gives the
same matrix.  Matrices are returned as CSR triplets (int32 rowptr, int32
colidx with sorted columns, float64 values) inside a small ``Instance``
record.

Workload shapes follow the paper's experiments (Sec. 4) and the benchmark
configurations of this project:

* ``givens_known``: A = G1 * D * G2 with D rectangular diagonal and G1/G2
  products of random Givens rotations, so the singular values are exactly
  the diagonal of D (used for the 1200 x 1000 plain FP64 case).
* ``model_problem``: Experiment II model problems 1 and 2 (Sec. 4.2,
  eqs. model1/model2): m = 1000, n = 200, A = U Sigma V^T with orthogonal
  factors from random matrices.
* ``random_sparse``: k distinct uniformly random rows per column, N(0,1)
  values (the large random and batched cases).
* ``zipf_rows``: row lengths drawn from a truncated Zipf law, columns uniform
  without replacement inside a row (power-law case).
* ``known_spectrum_sparse``: a sparse surrogate with a prescribed spectrum:
  D wrapped by two levels of disjoint random Givens rotations on rows and on
  columns, so exact singular values and vectors are known at large sizes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Instance", "rng_for", "givens_known", "model_problem", "random_sparse",
    "zipf_rows", "known_spectrum_sparse", "v_in", "csr_from_dense",
    "interval_by_count", "batch_pool", "serving_pool",
]


@dataclasses.dataclass
class Instance:
    """A sparse test matrix in CSR form plus what is known about it."""
    m: int
    n: int
    rowptr: np.ndarray          # int32 [m+1]
    colidx: np.ndarray          # int32 [nnz], sorted within each row
    vals: np.ndarray            # float64 [nnz]
    sigma: Optional[np.ndarray] = None   # exact singular values (descending) if known
    U: Optional[np.ndarray] = None       # exact left singular vectors (m x n) if known
    V: Optional[np.ndarray] = None       # exact right singular vectors (n x n) if known
    a: Optional[float] = None            # target interval, if the recipe fixes one
    b: Optional[float] = None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.vals.size)

    def dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n))
        for i in range(self.m):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            A[i, self.colidx[s:e]] = self.vals[s:e]
        return A

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.colidx, self.rowptr), shape=(self.m, self.n))


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2109, 13655, int(config), int(instance)]))


def csr_from_dense(A: np.ndarray, drop_zeros: bool = True):
    m, n = A.shape
    mask = A != 0.0 if drop_zeros else np.ones_like(A, dtype=bool)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    rows, cols = np.nonzero(mask)          # row-major order, columns ascending
    return (rowptr.astype(np.int32), cols.astype(np.int32), A[rows, cols].astype(np.float64))


def _csr_from_coo(m, n, rows, cols, vals):
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=m)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64)


def _rotate_rows(A, i, j, th):
    c, s = math.cos(th), math.sin(th)
    ri = A[i].copy()
    rj = A[j].copy()
    A[i] = c * ri - s * rj
    A[j] = s * ri + c * rj


def _rotate_cols(A, i, j, th):
    c, s = math.cos(th), math.sin(th)
    ci = A[:, i].copy()
    cj = A[:, j].copy()
    A[:, i] = c * ci - s * cj
    A[:, j] = s * ci + c * cj


def givens_known(m: int = 1200, n: int = 1000, sigma: Optional[np.ndarray] = None,
                 nrot: int = 2000, config: int = 1, instance: int = 0,
                 a: float = 0.40, b: float = 0.45) -> Instance:
    """A = G1 * D * G2 with exact singular values ``sigma``.

    G1 is a product of ``nrot`` rotations on random distinct row pairs of m,
    G2 a product of ``nrot`` rotations on random distinct column pairs of n,
    angles uniform in [0, 2 pi).  Left factor: U = G1[:, :n]; right factor:
    V = G2^T.  Returned sigma/U/V are sorted by descending sigma.
    """
    rng = rng_for(config, instance)
    if sigma is None:
        sigma = np.linspace(0.01, 1.0, n)
    sigma = np.asarray(sigma, dtype=np.float64)
    G1 = np.eye(m)
    G2 = np.eye(n)        # accumulates the column rotations: A = G1 D G2
    A = np.zeros((m, n))
    A[np.arange(n), np.arange(n)] = sigma
    for _ in range(nrot):
        i, j = rng.choice(m, 2, replace=False)
        th = rng.uniform(0.0, 2.0 * math.pi)
        _rotate_rows(A, i, j, th)
        _rotate_rows(G1, i, j, th)
    for _ in range(nrot):
        i, j = rng.choice(n, 2, replace=False)
        th = rng.uniform(0.0, 2.0 * math.pi)
        # right-multiply A by a rotation acting on columns i, j
        _rotate_cols(A, i, j, th)
        _rotate_cols(G2, i, j, th)
    # A = G1 D G2, so A G2^T = G1 D: the right singular vectors are the
    # columns of G2^T and the left ones the first n columns of G1.
    order = np.argsort(-sigma, kind="stable")
    rp, ci, va = csr_from_dense(A)
    return Instance(m, n, rp, ci, va, sigma=sigma[order], U=G1[:, :n][:, order],
                    V=G2.T[:, order], a=a, b=b, name=f"givens_{m}x{n}")


def model_problem(kind: int, instance: int = 0) -> Instance:
    """Experiment II model problems (m = 1000, n = 200).

    kind 1: singular values 0.005, 0.015, ..., 1.995 (uniform), target [0.8, 1.2].
    kind 2: singular values 10^-10, 10^-9.95, ..., 10^-0.05 (log-uniform),
            target [1e-3, 1e-1].
    U and V are orthogonal factors of Gaussian random matrices.
    """
    m, n = 1000, 200
    rng = rng_for(100 + kind, instance)
    if kind == 1:
        sigma = 0.005 + 0.01 * np.arange(n)
        a, b = 0.8, 1.2
    elif kind == 2:
        sigma = 10.0 ** (-10.0 + 0.05 * np.arange(n))
        a, b = 1e-3, 1e-1
    else:
        raise ValueError("kind must be 1 or 2")
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (U * sigma) @ V.T
    order = np.argsort(-sigma, kind="stable")
    rp, ci, va = csr_from_dense(A, drop_zeros=False)
    return Instance(m, n, rp, ci, va, sigma=sigma[order], U=U[:, order], V=V[:, order],
                    a=a, b=b, name=f"model{kind}")


def random_sparse(m: int, n: int, nnz_per_col: int, config: int = 2, instance: int = 0,
                  rng: Optional[np.random.Generator] = None) -> Instance:
    """k distinct uniform rows per column, N(0,1) values, CSR float64."""
    if rng is None:
        rng = rng_for(config, instance)
    k = int(nnz_per_col)
    # distinct rows per column: sample with rejection of duplicates per column
    rows = rng.integers(0, m, size=(n, k), dtype=np.int64)
    rows.sort(axis=1)
    dup = np.zeros_like(rows, dtype=bool)
    dup[:, 1:] = rows[:, 1:] == rows[:, :-1]
    while dup.any():
        rows[dup] = rng.integers(0, m, size=int(dup.sum()), dtype=np.int64)
        rows.sort(axis=1)
        dup[:] = False
        dup[:, 1:] = rows[:, 1:] == rows[:, :-1]
    cols = np.repeat(np.arange(n, dtype=np.int64), k)
    vals = rng.standard_normal(n * k)
    rp, ci, va = _csr_from_coo(m, n, rows.ravel(), cols, vals)
    return Instance(m, n, rp, ci, va, name=f"rand_{m}x{n}_k{k}")


def zipf_rows(m: int, n: int, alpha: float = 1.8, kmax: int = 42207, config: int = 5,
              instance: int = 0) -> Instance:
    """Row lengths iid truncated Zipf(alpha) on 1..kmax; columns uniform without
    replacement inside each row; N(0,1) values."""
    rng = rng_for(config, instance)
    ks = np.arange(1, kmax + 1, dtype=np.float64)
    p = ks ** (-alpha)
    p /= p.sum()
    lens = rng.choice(np.arange(1, kmax + 1), size=m, p=p).astype(np.int64)
    lens = np.minimum(lens, n)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    nnz = int(rowptr[-1])
    colidx = np.empty(nnz, dtype=np.int32)
    for i in range(m):
        s, e = rowptr[i], rowptr[i + 1]
        L = e - s
        if L * 8 < n:
            c = np.unique(rng.integers(0, n, size=L + 8))
            while c.size < L:
                c = np.unique(np.concatenate([c, rng.integers(0, n, size=L)]))
            c = rng.permutation(c)[:L]
            c.sort()
        else:
            c = np.sort(rng.choice(n, size=L, replace=False))
        colidx[s:e] = c
    vals = rng.standard_normal(nnz)
    if rowptr[-1] >= 2 ** 31:
        raise ValueError("nnz exceeds int32 CSR range")
    return Instance(m, n, rowptr.astype(np.int32), colidx, vals, name=f"zipf_{m}x{n}")


def known_spectrum_sparse(m: int, n: int, sigma: np.ndarray, levels: int = 2,
                          config: int = 20, instance: int = 0) -> Instance:
    """Sparse matrix with exactly the singular values ``sigma`` (length n).

    D (m x n, diag sigma) is wrapped by ``levels`` rounds of disjoint Givens
    rotations on random row pairs and on random column pairs.  Each round
    rotates a random perfect matching of the indices, so every row/column gets
    at most 2^levels nonzeros from the diagonal, and the singular vectors are
    known products of rotations (not returned: only sigma is kept).
    """
    rng = rng_for(config, instance)
    sigma = np.asarray(sigma, dtype=np.float64)
    # sparse representation as dict-of-rows would be slow; use COO and apply
    # rotations as small sparse products with scipy.
    import scipy.sparse as sp
    A = sp.csr_matrix((sigma, (np.arange(n), np.arange(n))), shape=(m, n))

    def rot_matrix(size):
        perm = rng.permutation(size)
        half = size // 2
        i, j = perm[:half], perm[half:2 * half]
        th = rng.uniform(0.0, 2.0 * math.pi, size=half)
        c, s = np.cos(th), np.sin(th)
        rows = np.concatenate([i, i, j, j])
        cols = np.concatenate([i, j, i, j])
        vals = np.concatenate([c, -s, s, c])
        if size % 2:
            k = perm[-1:]
            rows = np.concatenate([rows, k]); cols = np.concatenate([cols, k]); vals = np.concatenate([vals, [1.0]])
        return sp.csr_matrix((vals, (rows, cols)), shape=(size, size))

    for _ in range(levels):
        A = rot_matrix(m) @ A
    for _ in range(levels):
        A = A @ rot_matrix(n)
    A = A.tocsr()
    A.sort_indices()
    A.eliminate_zeros()
    return Instance(m, n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                    A.data.astype(np.float64), sigma=np.sort(sigma)[::-1],
                    name=f"known_{m}x{n}")


def v_in(n: int, L: int, config: int = 0, instance: int = 0, stream: int = 7) -> np.ndarray:
    """N(0,1) float64 block, n x L, Fortran (column-major) order."""
    rng = np.random.default_rng(np.random.SeedSequence([2109, 13655, int(config), int(instance), int(stream)]))
    return np.asfortranarray(rng.standard_normal((n, L)))


def interval_by_count(eigs_sq: np.ndarray, center_index: int, count: int):
    """Interval [a, b] on singular values whose squared end points sit at the
    midpoints between consecutive eigenvalues of A^T A, so that exactly
    ``count`` eigenvalues (ascending array ``eigs_sq``) fall inside."""
    ev = np.sort(np.asarray(eigs_sq, dtype=np.float64))
    lo = int(center_index) - count // 2
    hi = lo + count
    lo = max(lo, 1)
    hi = min(hi, ev.size - 1)
    a2 = 0.5 * (ev[lo - 1] + ev[lo])
    b2 = 0.5 * (ev[hi - 1] + ev[hi])
    return math.sqrt(max(a2, 0.0)), math.sqrt(b2)


def batch_pool(count: int = 64, m_lo: int = 5000, m_hi: int = 50000, config: int = 3):
    """Independent random sparse instances for the batched case: m uniform in
    [m_lo, m_hi], n = m // 2, 8..16 nonzeros per column, N(0,1) values, each with
    an interval of 16..32 eigenvalues of A^T A around the median (exact counts
    from a dense eigensolver, feasible for the sizes used in tests)."""
    rng = rng_for(config, 0)
    out = []
    for i in range(count):
        m = int(rng.integers(m_lo, m_hi + 1))
        n = m // 2
        k = int(rng.integers(8, 17))
        t = int(rng.integers(16, 33))
        inst = random_sparse(m, n, k, config=config, instance=1000 + i)
        inst.name = f"batch{i}_{m}x{n}_k{k}"
        out.append((inst, t))
    return out


def serving_pool(count: int = 32, n_lo: float = 1e4, n_hi: float = 3e5, config: int = 4):
    """Matrices for the serving case: n log-uniform in [n_lo, n_hi], m = 1.5 n,
    12 nonzeros per column, N(0,1) values."""
    rng = rng_for(config, 0)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(round(1.5 * n))
        inst = random_sparse(m, n, 12, config=config, instance=1000 + i)
        inst.name = f"serve{i}_{m}x{n}"
        out.append(inst)
    return out


def splitmix_normal(seed: int, n: int, L: int) -> np.ndarray:
    """N(0,1) block (n x L, column-major) from the counter-based generator the
    GPU library uses when it is given no V_in: SplitMix64 (Steele, Lea and
    Flood, 2014), output k of the stream seeded with s being
    mix(s + (k+1) * 0x9E3779B97F4A7C15); entry e (column-major) takes outputs
    2e and 2e+1 as u1, u2 = top 53 bits / 2^53 and the Box-Muller value
    sqrt(-2 ln(1 - u1)) cos(2 pi u2)."""
    M64 = (1 << 64) - 1
    g = 0x9E3779B97F4A7C15

    def mix(z):
        z = z & M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & M64
        return z ^ (z >> np.uint64(31))

    count = n * L
    e = np.arange(count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        k1 = np.uint64(2) * e
        z1 = np.uint64(seed) + (k1 + np.uint64(1)) * np.uint64(g)
        z2 = np.uint64(seed) + (k1 + np.uint64(2)) * np.uint64(g)
        u1 = (mix(z1) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        u2 = (mix(z2) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    x = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    return np.asfortranarray(x.reshape(L, n).T)


def interval_from_sample(m: int, n: int, nnz_per_col: int, count: int, scale: int = 25, config: int = 2,
                         quantile: float = 0.5):
    """Interval [a, b] expected to hold about ``count`` singular values of a
    random sparse m x n matrix (k nonzeros per column, N(0,1)) around the
    ``quantile`` of its spectrum.

    The spectrum is read off a same-distribution instance of size
    (m/scale) x (n/scale): dense eigenvalues of its A^T A give the quantile
    lambda_q and the local eigenvalue density (eigenvalues per unit lambda in
    a window of 5% of the spectrum around lambda_q); the full-size density is
    ``scale`` times larger, so the interval in lambda is count / (scale *
    density) wide.  Returns (a, b, lambda_q, density)."""
    ms, ns = max(m // scale, 2), max(n // scale, 1)
    I = random_sparse(ms, ns, nnz_per_col, config=config, instance=99)
    A = I.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    lq = float(np.quantile(ev, quantile))
    w = 0.05 * (ev[-1] - ev[0])
    dens = np.sum(np.abs(ev - lq) <= w / 2) / w
    width = count / (scale * dens)
    return math.sqrt(lq - width / 2), math.sqrt(lq + width / 2), lq, dens


def sample_spectrum(m: int, n: int, nnz_per_col: int, scale: int = 25, config: int = 2) -> np.ndarray:
    """n singular values (descending) distributed like those of a random
    sparse m x n matrix with k nonzeros per column: the eigenvalues of A^T A
    of a same-distribution instance (m/scale) x (n/scale) define an empirical
    quantile function, read at the n midpoints (i + 1/2)/n.  Used as the
    exact spectrum of a known-spectrum surrogate of that matrix."""
    ms, ns = max(m // scale, 2), max(n // scale, 1)
    I = random_sparse(ms, ns, nnz_per_col, config=config, instance=99)
    A = I.dense()
    ev = np.sort(np.linalg.eigvalsh(A.T @ A))
    q = (np.arange(n) + 0.5) / n
    lam = np.interp(q, (np.arange(ns) + 0.5) / ns, ev)
    return np.sqrt(np.maximum(lam, 0.0))[::-1].copy()


def interval_from_zipf_sample(m: int, n: int, count: int, scale: int = 200, config: int = 5,
                              quantile: float = 0.5):
    """The recipe of ``interval_from_sample`` for Zipf-row matrices
    (``zipf_rows``): a same-distribution instance (m/scale) x (n/scale)
    (row lengths still truncated at 42,207, then capped at its n), dense
    eigenvalues of its A^T A for the quantile and the local density, scaled
    by ``scale`` to hold about ``count`` values.  Returns (a, b, lambda_q,
    density)."""
    ms, ns = max(m // scale, 2), max(n // scale, 1)
    I = zipf_rows(ms, ns, config=config, instance=99)
    A = I.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    lq = float(np.quantile(ev, quantile))
    w = 0.05 * (ev[-1] - ev[0])
    dens = np.sum(np.abs(ev - lq) <= w / 2) / w
    width = count / (scale * dens)
    return math.sqrt(max(lq - width / 2, 0.0)), math.sqrt(lq + width / 2), lq, dens
