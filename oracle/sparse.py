"""Plain CSR helpers (TEST INFRASTRUCTURE).

Definitions only: the transpose of a CSR matrix lists, for every column j of
A, the entries (i, a_ij) in increasing row order; the product y = A x is
y_i = sum_k a_{i, c_k} x_{c_k}.  Written with explicit loops over rows so a
reader can check them by eye; meant for small and sampled cases.
"""
from __future__ import annotations

import numpy as np


def transpose(m, n, rowptr, colidx, vals):
    cols = [[] for _ in range(n)]
    for i in range(m):
        for k in range(rowptr[i], rowptr[i + 1]):
            cols[colidx[k]].append((i, vals[k]))
    rp = np.zeros(n + 1, dtype=np.int64)
    ci, va = [], []
    for j in range(n):
        ent = sorted(cols[j])
        rp[j + 1] = rp[j] + len(ent)
        ci.extend(e[0] for e in ent)
        va.extend(e[1] for e in ent)
    return rp, np.array(ci, dtype=np.int64), np.array(va, dtype=np.float64)


def product_rows(rowptr, colidx, vals, X, rows):
    """Rows ``rows`` of A X for a dense X (n x k), one row at a time."""
    out = np.zeros((len(rows), X.shape[1]))
    for r, i in enumerate(rows):
        s, e = rowptr[i], rowptr[i + 1]
        out[r] = vals[s:e] @ X[colidx[s:e]]
    return out
