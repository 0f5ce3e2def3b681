"""Quadrature points, weights and filter functions (TEST INFRASTRUCTURE).

Definitions followed (paper Sec. 4, opening paragraphs of the experiments):
the N quadrature points lie on an ellipse with centre gamma, semi-axis rho
and aspect ratio alpha,

    theta_j = (2 pi / N) (j - 1/2),               j = 1..N
    z_j     = gamma + rho (cos theta_j + i alpha sin theta_j)
    omega_j = (rho / N) (alpha cos theta_j + i sin theta_j)
    psi_j   = (rho / N) exp(t_j) (alpha cos theta_j + i sin theta_j)

with (gamma, rho) = ((a^2+b^2)/2, (b^2-a^2)/2) for Algorithm 1 and
(gamma, rho) = (log a + log b, log b - log a) for Algorithm 2, where the
points are t_j and the shifts are g(t_j) = exp(t_j).

The filter functions are those of Sec. 3.2 (f) and Sec. 3.3 (f_g):

    f(sigma)   = sum_{j=1}^{N} omega_j / (z_j - sigma^2)
    f_g(sigma) = sum_{j=1}^{N} psi_j / (g(t_j) - sigma^2)
"""
from __future__ import annotations

import numpy as np

PLAIN = 0
EXP = 1


def ellipse(a: float, b: float, N: int, alpha: float = 0.1, transform: int = PLAIN):
    """All N points of the rule.

    Returns (theta, t, shift, weight): ``t`` are the contour points (z_j for
    the plain method, t_j for the transformed one), ``shift`` the matrix
    shifts (z_j, or exp(t_j)), ``weight`` the weights (omega_j or psi_j).
    """
    if N < 2 or N % 2:
        raise ValueError("N must be even and >= 2")
    if not (0.0 <= a < b):
        raise ValueError("need 0 <= a < b")
    j = np.arange(1, N + 1, dtype=np.float64)
    theta = 2.0 * np.pi / N * (j - 0.5)
    if transform == PLAIN:
        gamma = 0.5 * (a * a + b * b)
        rho = 0.5 * (b * b - a * a)
    elif transform == EXP:
        if a <= 0.0:
            raise ValueError("the exp transform needs a > 0 (log a)")
        gamma = np.log(a) + np.log(b)
        rho = np.log(b) - np.log(a)
    else:
        raise ValueError("unknown transform")
    t = gamma + rho * (np.cos(theta) + 1j * alpha * np.sin(theta))
    dir_ = alpha * np.cos(theta) + 1j * np.sin(theta)
    if transform == PLAIN:
        shift = t
        weight = rho / N * dir_
    else:
        shift = np.exp(t)
        weight = rho / N * np.exp(t) * dir_
    return theta, t, shift, weight


def half_rule(a, b, N, alpha=0.1, transform=PLAIN):
    """The upper-half points j = 1..N/2 (theta in (0, pi)).

    With theta_j = 2 pi (j - 1/2) / N the conjugate partner of point j is
    point N + 1 - j (Sec. 3.1, symmetry of the rule about the real axis), so
    the first N/2 points carry one member of every conjugate pair.
    """
    theta, t, shift, weight = ellipse(a, b, N, alpha, transform)
    h = N // 2
    return theta[:h], t[:h], shift[:h], weight[:h]


def moment_coeffs(a, b, N, M, alpha=0.1, transform=PLAIN):
    """c[j, k] = omega_j z_j^k (plain) or psi_j t_j^k (exp), j = 1..N/2,
    k = 0..M (Algorithm 1 / 2, step 2; one extra moment k = M is kept for
    the practical residual estimate of Sec. 3.4.1)."""
    _, t, shift, weight = half_rule(a, b, N, alpha, transform)
    k = np.arange(M + 1)
    c = weight[:, None] * t[:, None] ** k[None, :]
    return shift, c


def filter_f(sigma, a, b, N, alpha=0.1, transform=PLAIN):
    """f(sigma) (plain) or f_g(sigma) (exp) summed over all N points."""
    _, _, shift, weight = ellipse(a, b, N, alpha, transform)
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    return (weight[None, :] / (shift[None, :] - s2.reshape(-1, 1))).sum(axis=1).reshape(np.shape(sigma))
