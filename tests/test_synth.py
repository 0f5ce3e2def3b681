"""The seeded generators reproduce the spectra their recipes promise."""
import numpy as np

import synth


def test_givens_exact_spectrum_and_vectors():
    I = synth.givens_known(300, 250, nrot=500)
    A = I.dense()
    assert np.abs(A @ I.V - I.U * I.sigma).max() < 1e-13
    assert np.abs(np.linalg.svd(A, compute_uv=False) - I.sigma).max() < 1e-13
    # CSR well formed: monotone rowptr, sorted in-range columns
    assert np.all(np.diff(I.rowptr) >= 0) and I.rowptr[-1] == I.nnz
    for i in range(I.m):
        c = I.colidx[I.rowptr[i]:I.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0) and (c.size == 0 or (c[0] >= 0 and c[-1] < I.n))


def test_givens_deterministic():
    a, b = synth.givens_known(120, 100, nrot=100), synth.givens_known(120, 100, nrot=100)
    assert np.array_equal(a.vals, b.vals) and np.array_equal(a.colidx, b.colidx)


def test_random_sparse_column_counts():
    I = synth.random_sparse(500, 200, 9, config=60)
    cols = np.bincount(I.colidx, minlength=200)
    assert np.all(cols == 9)
    S = I.scipy()
    assert S.nnz == 1800


def test_known_spectrum_sparse():
    sig = np.linspace(0.1, 2.0, 300)
    I = synth.known_spectrum_sparse(500, 300, sig)
    s = np.linalg.svd(I.dense(), compute_uv=False)
    assert np.abs(s - np.sort(sig)[::-1]).max() < 1e-13
    assert np.diff(I.rowptr).max() <= 4 * 1 + 0 or np.diff(I.rowptr).max() <= 16


def test_zipf_rows_small():
    I = synth.zipf_rows(2000, 1000, kmax=500, config=61)
    lens = np.diff(I.rowptr)
    assert lens.min() >= 1 and lens.max() <= 500
    for i in range(0, 2000, 97):
        c = I.colidx[I.rowptr[i]:I.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_model_problems():
    for k in (1, 2):
        I = synth.model_problem(k)
        A = I.dense()
        assert np.abs(A @ I.V - I.U * I.sigma).max() < 1e-14
