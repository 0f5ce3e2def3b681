"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage or the mathematical fact it relies on.  None of
them retypes the oracle's own formula: they compare it with closed forms,
exact spectra, invariants, a second independent solver, or numbers printed in
the paper (``tests/golden/paper_values.json``).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import krylov, method, quadrature as Q, truth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ---------------------------------------------------------------- quadrature

@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_circle_closed_form(N):
    """For alpha = 1 the N-point trapezoid rule on a circle gives the rational
    filter f(lambda) = 1 / (1 + x^N), x = (lambda - gamma)/rho (geometric
    series of the discrete Fourier sum); hence f = 1/2 at both end points."""
    a, b = 0.3, 0.7
    gamma, rho = (a * a + b * b) / 2, (b * b - a * a) / 2
    s = np.linspace(0.0, 1.2, 97)
    x = (s * s - gamma) / rho
    f = Q.filter_f(s, a, b, N, alpha=1.0)
    np.testing.assert_allclose(f.real, 1.0 / (1.0 + x ** N), atol=1e-13)
    assert np.abs(f.imag).max() < 1e-13
    fe = Q.filter_f(np.array([a, b]), a, b, N, alpha=1.0)
    np.testing.assert_allclose(fe.real, [0.5, 0.5], atol=1e-13)


@pytest.mark.parametrize("transform", [Q.PLAIN, Q.EXP])
@pytest.mark.parametrize("N", [8, 16, 32])
def test_quadrature_condition(N, transform):
    """eq. cond: sum_j w_j p(t_j) = 0 for every polynomial of degree <= N-2
    (trapezoid rule exact for trigonometric polynomials of degree < N), and
    not for degree N-1.  Checked in the scale-free variable x = (t-gamma)/rho;
    for the exp transform the weights are psi_j / exp(t_j) (dt-measure)."""
    a, b, alpha = 0.2, 0.9, 0.1
    theta, t, shift, w = Q.ellipse(a, b, N, alpha, transform)
    if transform == Q.PLAIN:
        gamma, rho = (a * a + b * b) / 2, (b * b - a * a) / 2
    else:
        gamma, rho = np.log(a) + np.log(b), np.log(b) - np.log(a)
        w = w / np.exp(t)
    x = (t - gamma) / rho
    for k in range(N - 1):
        scale = np.sum(np.abs(w) * np.abs(x) ** k)
        assert abs(np.sum(w * x ** k)) <= 1e-14 * scale
    # degree N-1: the e^{iN theta} term survives; its relative size is
    # ((1 - alpha)/2)^(N-1)-like, far above the rounding level checked above
    k = N - 1
    scale = np.sum(np.abs(w) * np.abs(x) ** k)
    assert abs(np.sum(w * x ** k)) >= 1e-8 * scale


def test_conjugate_pairing_and_halving():
    """Sec. 3.1 symmetry: point N+1-j is the conjugate of point j (with
    theta_j = 2 pi (j-1/2)/N), and the full N-point moment sum equals twice
    the real part of the half sum (its imaginary part vanishes)."""
    a, b, N = 0.4, 0.45, 16
    _, t, shift, w = Q.ellipse(a, b, N)
    np.testing.assert_allclose(t[::-1], np.conj(t), rtol=0, atol=1e-15)
    np.testing.assert_allclose(w[::-1], np.conj(w), rtol=0, atol=1e-15)
    I = synth.givens_known(120, 100, nrot=300, a=a, b=b)
    A = I.dense()
    G = A.T @ A
    V = synth.v_in(I.n, 4, 1)
    Yfull = method.shifted_solves(G, shift, V)
    M = 3
    full = np.stack([sum(w[j] * t[j] ** k * Yfull[j] for j in range(N)) for k in range(M)])
    half, _, _, _ = method.filtered_moments(A, a, b, V, M - 1, N, G=G)
    assert np.abs(full.imag).max() <= 1e-12 * np.abs(full.real).max()
    np.testing.assert_allclose(half, full.real, rtol=0, atol=1e-12 * np.abs(full.real).max())


# ------------------------------------------------------------------ moments

def test_prop1_powers_of_gram():
    """Proposition 1: S_k = (A^T A)^k S_0 for k <= N-1 (plain rule)."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((60, 40)) / 8
    G = A.T @ A
    ev = np.linalg.eigvalsh(G)
    a, b = np.sqrt(ev[18] * 0.5 + ev[17] * 0.5), np.sqrt(ev[26] * 0.5 + ev[27] * 0.5)
    V = rng.standard_normal((40, 3))
    S, _, _, _ = method.filtered_moments(A, a, b, V, 5, 16, G=G)
    for k in range(1, 6):
        ref = np.linalg.matrix_power(G, k) @ S[0]
        assert np.abs(S[k] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("transform", [Q.PLAIN, Q.EXP])
def test_moments_spectral_form(transform):
    """Thm 1 proof / Prop 1 expansion: with A = U Sigma V^T,
    S_k = V diag(h_k(sigma)) V^T V_in, h_k(s) = sum_j c_jk / (shift_j - s^2)
    summed over all N points; for the plain rule h_k(s) = s^{2k} f(s).
    The oracle gets S_k from linear solves; here it is rebuilt from the
    exact singular vectors of the generator."""
    a, b, N, M = 0.4, 0.45, 16, 4
    sig = np.linspace(0.05, 1.0, 80)
    I = synth.givens_known(100, 80, sigma=sig, nrot=400, a=a, b=b)
    V_in = synth.v_in(I.n, 5, 2)
    S, _, _, _ = method.filtered_moments(I, a, b, V_in, M, N, transform=transform)
    _, t, shift, w = Q.ellipse(a, b, N, 0.1, transform)
    coef = I.V.T @ V_in
    for k in range(M + 1):
        h = np.array([np.sum(w * t ** k / (shift - s * s)) for s in I.sigma])
        assert np.abs(h.imag).max() < 1e-12
        if transform == Q.PLAIN:
            f = Q.filter_f(I.sigma, a, b, N)
            np.testing.assert_allclose(h.real, I.sigma ** (2 * k) * f.real, rtol=1e-9, atol=1e-15)
        ref = I.V @ (h.real[:, None] * coef)
        assert np.abs(S[k] - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())


def test_exp_weights_include_derivative():
    """Alg. 2 weights psi_j carry g'(t_j) = exp(t_j), so f_g ~ 1 inside
    [a, b] and ~ 0 far outside (residue of exp(t)/(exp(t)-s^2) at
    t = log s^2 is 1)."""
    a, b = 0.01, 0.1
    fg = Q.filter_f(np.array([0.03162, 1e-5, 10.0]), a, b, 32, transform=Q.EXP)
    assert abs(fg[0] - 1.0) < 0.1
    assert abs(fg[1]) < 1e-6 and abs(fg[2]) < 1e-6


def test_exp1_filter_shapes():
    """Experiment I (Sec. 4.1, Fig. 1): for [1e-3, 1e-1] the plain filter is
    about 0.5 for tiny sigma, while f_g drops sharply; for [0.8, 1.2] both
    filters agree closely."""
    g = GOLD["exp1"]
    a, b = g["interval"]
    tiny = np.array([1e-6, 1e-5, 1e-4])
    f = np.abs(Q.filter_f(tiny, a, b, 32))
    fg = np.abs(Q.filter_f(tiny, a, b, 32, transform=Q.EXP))
    assert np.all(np.abs(f - g["f_below_a_approx"]) < 0.05)
    assert np.all(fg < 1e-12)
    s = np.linspace(0.5, 1.5, 41)
    f1 = np.abs(Q.filter_f(s, 0.8, 1.2, 32))
    f2 = np.abs(Q.filter_f(s, 0.8, 1.2, 32, transform=Q.EXP))
    assert np.abs(f1 - f2).max() < 0.15


# ------------------------------------------------------- end-to-end method

def _run(I, L, M, N, transform=Q.PLAIN, ell=1, eps=1e-12):
    V = synth.v_in(I.n, L, 9)
    return method.ss_svd(I, I.a, I.b, V, L, M, N, ell=ell, transform=transform, eps=eps)


def test_model1_exact_sigma():
    """Experiment II model problem 1 (eq. model1) with (L,M,N,ell,delta) of
    Sec. 4.2: the 40 singular values in [0.8, 1.2] are recovered to the FP64
    accuracy level of Table 2."""
    p = GOLD["exp2_parameters"]
    I = synth.model_problem(1)
    out = _run(I, p["L"], p["M"], p["N"])
    exact = np.sort(I.sigma[(I.sigma >= 0.8) & (I.sigma <= 1.2)])
    assert exact.size == GOLD["exp2_model1"]["count"]
    assert out["sigma"].size == exact.size
    rel = np.abs(out["sigma"] - exact) / exact
    acc = GOLD["exp3_table2_accuracy"]
    assert rel.max() <= 10 * acc["max_error"]
    res = truth.triplet_residuals(I, out["sigma"], out["U"], out["V"], normA=I.sigma[0])
    assert res.max() <= 10 * acc["max_residual"]


def test_model2_transform_beats_plain():
    """Sec. 4.2, Fig. 2(b): on the log-uniform model problem 2 the exp
    transform (Alg. 2) is far more accurate than the plain method (Alg. 1)."""
    p = GOLD["exp2_parameters"]
    I = synth.model_problem(2)
    exact = np.sort(I.sigma[(I.sigma >= I.a) & (I.sigma <= I.b)])
    o_nt = _run(I, p["L"], p["M"], p["N"], transform=Q.EXP)
    o_pl = _run(I, p["L"], p["M"], p["N"], transform=Q.PLAIN)
    assert o_nt["sigma"].size == exact.size
    rel_nt = np.abs(o_nt["sigma"] - exact) / exact
    res_nt = truth.triplet_residuals(I, o_nt["sigma"], o_nt["U"], o_nt["V"], normA=I.sigma[0])
    assert rel_nt.max() < 1e-9 and res_nt.max() < 1e-10
    res_pl = truth.triplet_residuals(I, o_pl["sigma"], o_pl["U"], o_pl["V"], normA=I.sigma[0])
    assert res_pl.max() > 1e3 * res_nt.max()


def test_givens_1200x1000_interval():
    """Plain FP64 case A = G1 D G2 (1200 x 1000, sigma = linspace(0.01, 1, 1000)),
    [0.40, 0.45], N=16, L=16, M=8: 50 strict-interior singular values plus
    one edge value (the 445th linspace point equals 0.45 up to rounding).  At
    ell = 1 the method itself limits the residual (~1e-6: the 50-dimensional
    target space is reached only through high moments); ell = 2 (eq. iter1)
    squares the filter and reaches <= 1e-8."""
    I = synth.givens_known()
    strict, edge = truth.strict_count(I.sigma, I.a, I.b, 1e-12)
    assert (strict, edge) == (50, 1)
    for ell, bound in ((1, 5e-6), (2, 1e-8)):
        out = _run(I, 16, 8, 16, ell=ell)
        core = (out["sigma"] > I.a + 1e-12) & (out["sigma"] < I.b - 1e-12)
        assert core.sum() == 50
        exact = np.sort(I.sigma[(I.sigma > I.a + 1e-12) & (I.sigma < I.b - 1e-12)])
        assert np.abs(out["sigma"][core] - exact).max() < bound
        res = truth.triplet_residuals(I, out["sigma"], out["U"], out["V"], normA=1.0)
        assert res.max() < bound


def test_random_sparse_against_dense_truth():
    """Method (Alg. 1) against the dense LAPACK truth on a small random
    sparse matrix: same count in [a, b] and tiny residuals."""
    I = synth.random_sparse(600, 300, 8, config=50)
    A = I.dense()
    ev = np.linalg.eigvalsh(A.T @ A)
    I.a, I.b = synth.interval_by_count(ev, 150, 12)
    s, U, V, sall = truth.dense_truth(I, I.a, I.b)
    assert s.size == 12
    out = _run(I, 8, 4, 32)
    assert out["sigma"].size == 12
    np.testing.assert_allclose(out["sigma"], s, rtol=1e-10)
    res = truth.triplet_residuals(I, out["sigma"], out["U"], out["V"], normA=sall[0])
    assert res.max() < 1e-10
    for i in range(12):
        assert abs(abs(out["V"][:, i] @ V[:, i]) - 1.0) < 1e-8


def test_spurious_index_separates_noise():
    """Sec. 3.4.2: with delta = 1e-20 nothing is truncated, so Ritz values
    from noise directions of S-hat show up inside [a, b]; their tau is tiny
    and their residual large, while every kept triplet is accurate."""
    I = synth.model_problem(1)
    out = _run(I, 20, 4, 32, eps=0.0)
    res_all = truth.triplet_residuals(I, out["sigma"], out["U"], out["V"], normA=I.sigma[0])
    tau_rel = out["tau"] / out["sS"][0]
    bad = res_all > 1e-6
    assert bad.any()
    assert tau_rel[bad].max() < 1e-14
    assert tau_rel[~bad].min() > 1e-6


def test_residual_estimate_plain():
    """eq. residual: for Alg. 1 the estimate from S_+ equals the exact
    residual ||A^T u - sigma v|| (Prop 1 makes S_+ = A^T A S-hat).  A
    deliberately small subspace (L=14, N=16) keeps the residuals well above
    rounding so the comparison is meaningful."""
    I = synth.model_problem(1)
    out = _run(I, 14, 4, 16)
    A = I.dense()
    exact = np.linalg.norm(A.T @ out["U"] - out["V"] * out["sigma"], axis=0)
    assert exact.min() > 1e-8
    est = out["resid_est"]
    np.testing.assert_allclose(est, exact, rtol=1e-6)


def test_residual_estimate_exp_mu():
    """eq. res_nonlinear: for Alg. 2 the scaled estimate mu ||r~_i|| tracks
    the exact residuals (Fig. 4: 'well estimated') within a small factor."""
    I = synth.model_problem(2)
    out = _run(I, 20, 4, 32, transform=Q.EXP)
    A = I.dense()
    exact = np.linalg.norm(A.T @ out["U"] - out["V"] * out["sigma"], axis=0)
    mu = method.nt_mu(out["resid_est"], exact)
    ratio = mu * out["resid_est"] / exact
    assert np.all((ratio > 1e-2) & (ratio < 1e2))


def test_ell_iteration_squares_filter():
    """Sec. 3.1 eq. iter1/iter2: with ell rounds the moments are
    V diag(sigma^{2k} f(sigma)^ell) V^T V_in (expansion before eq. S=FK)."""
    a, b, N = 0.4, 0.45, 16
    sig = np.linspace(0.05, 1.0, 80)
    I = synth.givens_known(100, 80, sigma=sig, nrot=400, a=a, b=b)
    V_in = synth.v_in(I.n, 3, 4)
    S, _, _, _ = method.filtered_moments(I, a, b, V_in, 2, N, ell=2)
    f = Q.filter_f(I.sigma, a, b, N).real
    for k in range(3):
        ref = I.V @ ((I.sigma ** (2 * k) * f ** 2)[:, None] * (I.V.T @ V_in))
        assert np.abs(S[k] - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())


# ------------------------------------------------------------ other pieces

def test_cocg_matches_direct_solve():
    """The oracle's COCG (independent iterative solver) reproduces LAPACK's
    zgesv on a shifted system."""
    I = synth.random_sparse(300, 150, 6, config=51)
    A = I.dense()
    G = A.T @ A
    z = np.median(np.linalg.eigvalsh(G)) + 0.05j
    V = synth.v_in(150, 3, 5)
    Y, it, res, _ = krylov.cocg(I, z, V, tol=1e-12, maxit=5000)
    ref = np.linalg.solve(z * np.eye(150) - G, V.astype(complex))
    assert res.max() <= 1e-12
    assert np.abs(Y - ref).max() <= 1e-8 * np.abs(ref).max()


def test_table1_subspace_rule():
    """Table 1: M = 4 and L chosen so that L M ~ 3 t."""
    for row in GOLD["exp3_table1"]["rows"]:
        assert row["M"] == 4
        assert abs(row["L"] * row["M"] - 3 * row["t"]) <= 0.25 * 3 * row["t"]


def test_model_counts_match_paper():
    """eq. model1/model2 spectra and the target counts of Sec. 4.2."""
    g1, g2 = GOLD["exp2_model1"], GOLD["exp2_model2"]
    I1, I2 = synth.model_problem(1), synth.model_problem(2)
    assert np.sum((I1.sigma >= 0.8) & (I1.sigma <= 1.2)) == g1["count"]
    strict, edge = truth.strict_count(I2.sigma, 1e-3, 1e-1, 1e-12)
    assert strict == 39 and edge == 2   # 41 in the closed interval; paper says 40
    assert abs(I1.sigma.min() - g1["sigma_first"]) < 1e-15
    assert abs(np.log10(I2.sigma.min()) - g2["log10_first"]) < 1e-12


def test_sparse_residual_certificate_matches_dense_definition():
    """The sparse certificate against the dense residuals on exact SVD
    triplets (both at rounding level), and a known answer: scaling v_i by
    (1 + e) makes both residuals of triplet i exactly e sigma_i ||v_i|| = e
    sigma_i, divided by ||A||_2 (a dropped term, a sign or a transposed
    operand breaks one of these)."""
    I = synth.random_sparse(300, 200, 5, config=91)
    Ad = I.dense()
    Uf, s, Vt = np.linalg.svd(Ad, full_matrices=False)
    sel = np.arange(40, 52)
    sig, U, V = s[sel], Uf[:, sel], Vt.T[:, sel].copy()
    nA = truth.norm2(Ad)
    rs = truth.sparse_triplet_residuals(I.rowptr, I.colidx, I.vals, I.m, I.n, sig, U, V, nA)
    rd = truth.triplet_residuals(Ad, sig, U, V, nA)
    assert rs.max() <= 1e-13 and rd.max() <= 1e-13
    eps = 1e-6
    V[:, 3] *= 1.0 + eps
    rs = truth.sparse_triplet_residuals(I.rowptr, I.colidx, I.vals, I.m, I.n, sig, U, V, nA)
    rd = truth.triplet_residuals(Ad, sig, U, V, nA)
    np.testing.assert_allclose(rs[3], eps * sig[3] / nA, rtol=1e-6)
    np.testing.assert_allclose(rs, rd, rtol=1e-9, atol=1e-15)
    assert np.delete(rs, 3).max() <= 1e-13


def test_sparse_norm_is_a_lower_bound():
    """The power-method estimate never exceeds ||A||_2 (LAPACK's SVD) and is
    close to it after enough steps."""
    I = synth.random_sparse(300, 200, 5, config=92)
    nA = truth.norm2(I.dense())
    est = truth.sparse_norm2_lower(I.rowptr, I.colidx, I.vals, I.m, I.n, iters=400)
    assert est <= nA * (1 + 1e-14)
    assert est >= nA * (1 - 1e-4)


def test_residual_estimate_exp_against_matrix_log():
    """eq. res_nonlinear, first factor: for Alg. 2 the unscaled estimate
    ||r~_i|| stands for (1/sigma_i) ||g^-1(A^T A) v_i - g^-1(sigma_i^2) v_i||
    with g^-1 = log (Sec. 3.4.1).  The matrix logarithm is formed here from
    the exactly known factors of model problem 2 (log(A^T A) = V diag(2 log
    sigma) V^T), not from the moments; the two agree to the accuracy of the
    exp-transformed moment relation on a deliberately small subspace (L = 10,
    N = 16) whose residuals sit far above rounding.  A missing factor 2 in
    g^-1(sigma^2), a dropped 1/sigma or the wrong singular vectors of S-hat
    each break the agreement by orders of magnitude."""
    I = synth.model_problem(2)
    out = method.ss_svd(I, I.a, I.b, synth.v_in(I.n, 10, 9), 10, 4, 16, transform=Q.EXP)
    v, s = out["V"], out["sigma"]
    assert s.size >= 30
    logG = (I.V * (2.0 * np.log(I.sigma))) @ I.V.T
    ref = np.linalg.norm(logG @ v - v * np.log(s ** 2)[None, :], axis=0) / s
    assert ref.min() > 1e-3  # far above rounding
    np.testing.assert_allclose(out["resid_est"], ref, rtol=1e-3)


def test_nt_mu_reproduces_the_chosen_exact_residual():
    """eq. res_nonlinear: mu = ||r_i'|| / ||r~_i'|| for one index i' taken from
    the exact residuals (the oracle takes the largest), so mu ||r~_i'|| equals
    ||r_i'|| exactly, and mu follows the estimates when every exact residual
    is scaled by one factor."""
    I = synth.model_problem(2)
    out = method.ss_svd(I, I.a, I.b, synth.v_in(I.n, 10, 9), 10, 4, 16, transform=Q.EXP)
    A = I.dense()
    exact = np.linalg.norm(A.T @ out["U"] - out["V"] * out["sigma"], axis=0)
    est = out["resid_est"]
    mu = method.nt_mu(est, exact)
    i = int(np.argmax(exact))
    assert mu * est[i] == pytest.approx(exact[i], rel=1e-15)
    assert method.nt_mu(est, 3.0 * exact) == pytest.approx(3.0 * mu, rel=1e-15)
    assert method.nt_mu(2.0 * est, exact) == pytest.approx(0.5 * mu, rel=1e-15)


def test_product_rows_against_dense_product():
    """oracle.sparse.product_rows is (A X)[rows] by definition: checked
    against the dense product on a matrix with empty rows, for all rows in
    order and for a shuffled sample with repeats."""
    from oracle import sparse
    rng = np.random.default_rng(77)
    m, n, k = 60, 45, 7
    A = rng.standard_normal((m, n)) * (rng.random((m, n)) < 0.15)
    A[[0, 13, 59]] = 0.0  # empty rows, including the first and the last
    rp, ci, va = synth.csr_from_dense(A)
    assert rp[1] == rp[0] and rp[14] == rp[13] and rp[-1] == rp[-2]
    X = rng.standard_normal((n, k))
    ref = A @ X
    got = sparse.product_rows(rp, ci, va, X, range(m))
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())
    assert np.all(got[[0, 13, 59]] == 0.0)
    rows = np.array([59, 3, 3, 40, 0, 22])
    np.testing.assert_allclose(sparse.product_rows(rp, ci, va, X, rows), ref[rows], rtol=1e-14,
                               atol=1e-14 * np.abs(ref).max())


def test_subspace_gap_known_principal_angles():
    """oracle.truth.subspace_gap is sin of the largest principal angle: two
    subspaces built from one orthonormal basis with known angles (0, theta1,
    theta2) give sin(max theta); the value does not depend on the bases
    chosen inside the subspaces; equal subspaces give 0 and orthogonal ones
    give 1."""
    rng = np.random.default_rng(78)
    n, k = 40, 3
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    th1, th2 = 0.3, 1.1
    X = Qm[:, :k]
    Y = np.column_stack([Qm[:, 0],
                         np.cos(th1) * Qm[:, 1] + np.sin(th1) * Qm[:, k],
                         np.cos(th2) * Qm[:, 2] + np.sin(th2) * Qm[:, k + 1]])
    assert truth.subspace_gap(X, Y) == pytest.approx(np.sin(th2), rel=1e-13)
    R1, _ = np.linalg.qr(rng.standard_normal((k, k)))
    R2, _ = np.linalg.qr(rng.standard_normal((k, k)))
    assert truth.subspace_gap(X @ R1, Y @ R2) == pytest.approx(np.sin(th2), rel=1e-12)
    assert truth.subspace_gap(X, X @ R1) <= 1e-14
    assert truth.subspace_gap(X, Qm[:, k:2 * k]) == pytest.approx(1.0, abs=1e-15)
    small = 1e-9  # tiny angles are resolved (the sine itself, not sqrt(1 - cos^2))
    Z = np.column_stack([Qm[:, 0], Qm[:, 1], np.cos(small) * Qm[:, 2] + np.sin(small) * Qm[:, k]])
    assert truth.subspace_gap(X, Z) == pytest.approx(small, rel=1e-5)
