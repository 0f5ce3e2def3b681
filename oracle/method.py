"""Algorithms 1 and 2 step by step with dense direct solves (TEST INFRASTRUCTURE).

Follows the paper's block SS-SVD method (Algorithm 1, Sec. 3.1) and its
variant with the nonlinear transformation g(t) = exp(t) (Algorithm 2,
Sec. 3.3), with the quadrature of Sec. 4 and the practical techniques of
Sec. 3.4 (residual estimate, eq. residual / eq. res_nonlinear; spurious
index tau).  Library primitives used as single steps: ``numpy.linalg.solve``
(LAPACK zgesv) for each shifted block system, ``numpy.linalg.svd`` (dgesdd)
and ``numpy.linalg.qr`` (dgeqrf, Householder).  No blocking, fusion or
reordering beyond what the algorithms state.

Readings of points the paper leaves open (listed with the design notes):
* delta is relative to the largest singular value of S-hat.
* the spurious test compares tau_i with eps * sigma_S,1 (tau has the units of
  a singular value of S-hat).
* the output keeps phi_i in the closed interval [a, b], ascending order,
  sign fixed so that the largest-magnitude entry of each v-hat is positive.
* the right singular vectors of S-hat used by eq. residual are W_S1.
"""
from __future__ import annotations

import numpy as np

from . import quadrature as Q


def as_dense(A):
    """Dense float64 copy of A (accepts an ndarray or a synth.Instance)."""
    if isinstance(A, np.ndarray):
        return np.asarray(A, dtype=np.float64)
    return A.dense()


def gram(A):
    """G = A^T A formed densely (the oracle never exploits sparsity)."""
    A = as_dense(A)
    return A.T @ A


def shifted_solves(G, shifts, R):
    """Y_j = (z_j I - A^T A)^{-1} R for every shift (Algorithm 1, steps 1-2)."""
    n = G.shape[0]
    I = np.eye(n)
    return np.stack([np.linalg.solve(z * I - G, R.astype(np.complex128)) for z in shifts])


def moment_sums(Y, c):
    """S_k = 2 sum_j Re(c_jk Y_j), k = 0..K-1, using the conjugate symmetry of
    the rule (Sec. 3.1): the N-point sum equals twice the real part of the
    sum over the upper-half points."""
    nshift, K = c.shape
    return np.stack([2.0 * np.real(sum(c[j, k] * Y[j] for j in range(nshift))) for k in range(K)])


def filtered_moments(A, a, b, V_in, M, N, ell=1, alpha=0.1, transform=Q.PLAIN, G=None):
    """Algorithm 1/2, steps 1-2.

    Step 1: S_0^(nu) = 2 sum_j Re(w_j (shift_j I - A^T A)^{-1} S_0^(nu-1)),
            nu = 1..ell-1, with S_0^(0) = V_in (eq. iter1).
    Step 2: S_k^(ell) = 2 sum_j Re(c_jk (shift_j I - A^T A)^{-1} S_0^(ell-1)),
            k = 0..M (eq. iter2; k = M is the extra moment of Sec. 3.4.1).

    Returns (moments [M+1, n, L], Y [N/2, n, L] of the last round, shifts, c).
    """
    if G is None:
        G = gram(A)
    shifts, c = Q.moment_coeffs(a, b, N, M, alpha, transform)
    R = np.asarray(V_in, dtype=np.float64)
    for _ in range(ell - 1):
        Y = shifted_solves(G, shifts, R)
        R = moment_sums(Y, c[:, :1])[0]
    Y = shifted_solves(G, shifts, R)
    S = moment_sums(Y, c)
    return S, Y, shifts, c


def block_S(S, M):
    """S-hat = [S_0, S_1, ..., S_{M-1}] (n x LM)."""
    return np.concatenate([S[k] for k in range(M)], axis=1)


def low_rank(Shat, delta):
    """Step 3: SVD of S-hat, keep singular values > delta * sigma_S,1."""
    Us, ss, Wst = np.linalg.svd(Shat, full_matrices=False)
    r = int(np.sum(ss > delta * ss[0])) if ss.size and ss[0] > 0 else 0
    return Us[:, :r], ss[:r], Wst[:r].T, ss


def spurious_index(q, sS1):
    """tau_i = q_i^T q_i / q_i^T Sigma_S1^{-1} q_i for every column q_i (Sec. 3.4.2)."""
    num = np.sum(q * q, axis=0)
    den = np.sum(q * q / sS1[:, None], axis=0)
    return num / den


def ss_svd(A, a, b, V_in, L, M, N, ell=1, delta=1e-20, alpha=0.1, transform=Q.PLAIN,
           eps=1e-12, G=None):
    """Algorithm 1 (transform=PLAIN) or Algorithm 2 (transform=EXP).

    Returns a dict with the selected triplets (ascending sigma), the tau
    values, the rank r of the low-rank step, the candidates before selection
    and the intermediate moments.
    """
    Ad = as_dense(A)
    V_in = np.asarray(V_in, dtype=np.float64)
    n = Ad.shape[1]
    if V_in.shape != (n, L):
        raise ValueError("V_in must be n x L")
    S, Y, shifts, c = filtered_moments(Ad, a, b, V_in, M, N, ell, alpha, transform, G)
    Shat = block_S(S, M)
    # Step 3: low-rank approximation, V~ = U_S1
    Us1, sS1, Ws1, sS_all = low_rank(Shat, delta)
    Vt = Us1
    # Step 4: [U~, B] = qr(A V~)
    Ut, B = np.linalg.qr(Ad @ Vt)
    # Step 5: SVD of B, triplets (phi_i, U~ p_i, V~ q_i)
    P, phi, Qt = np.linalg.svd(B)
    Qm = Qt.T
    tau = spurious_index(Qm, sS1)
    keep = (phi >= a) & (phi <= b) & (tau >= eps * sS1[0])
    idx = np.nonzero(keep)[0]
    idx = idx[np.argsort(phi[idx], kind="stable")]
    sig = phi[idx]
    U = Ut @ P[:, idx]
    V = Vt @ Qm[:, idx]
    for i in range(len(idx)):
        j = int(np.argmax(np.abs(V[:, i])))
        if V[j, i] < 0:
            V[:, i] = -V[:, i]
            U[:, i] = -U[:, i]
    # Sec. 3.4.1 residual estimate from S_+ = [S_1..S_M]
    Splus = np.concatenate([S[k] for k in range(1, M + 1)], axis=1)
    est = residual_estimate(Splus, Us1, sS1, Ws1, Qm[:, idx], sig, transform)
    return dict(sigma=sig, U=U, V=V, tau=tau[idx], r=Us1.shape[1], phi_all=phi, tau_all=tau,
                sS=sS_all, S=S, Y=Y, shifts=shifts, c=c, Shat=Shat, B=B, resid_est=est,
                Vtilde=Vt, Utilde=Ut)


def residual_estimate(Splus, Us1, sS1, Ws1, q, sig, transform=Q.PLAIN):
    """Sec. 3.4.1.

    Plain (eq. residual):
        ||r_i|| = (1/sigma_i) || S_+ W_S1 Sigma_S1^{-1} q_i - sigma_i^2 U_S1 q_i ||.
    Exp transform: the same expression with g^{-1}(sigma_i^2) = 2 log sigma_i
    in place of sigma_i^2 gives ||r~_i||, to be scaled by mu (eq.
    res_nonlinear), which needs one exact residual; this function returns the
    unscaled ||r~_i||.
    """
    if len(sig) == 0:
        return np.zeros(0)
    T = Splus @ (Ws1 @ (q / sS1[:, None]))
    lam = sig ** 2 if transform == Q.PLAIN else np.log(sig ** 2)
    R = T - (Us1 @ q) * lam[None, :]
    return np.linalg.norm(R, axis=0) / sig


def nt_mu(est_tilde, exact):
    """mu = ||r_i'|| / ||r~_i'|| from one exact residual (eq. res_nonlinear)."""
    i = int(np.argmax(exact))
    return exact[i] / est_tilde[i]
