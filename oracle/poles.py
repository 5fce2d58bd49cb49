"""Oracle: pole expansion of A^{-1/2} for the Gibbs refresh of phi (FP64, CPU).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Definitions followed (paper section / equation):
  * phi | theta ~ N(0, A^{-1}); phi = A^{-1/2} xi with xi ~ N(0, I)            (Section 3.1)
  * A^{-1/2} ≈ sum_p w_p (A + lambda_p I)^{-1}, lambda_p >= 0                  (eq. pex)
  * Appendix A, eq. (msqdisc): with m <= lambda_min(A), M >= lambda_max(A), k = sqrt(m/M),
    K = K(k^2), K' = K(1-k^2), w(t) = sqrt(m) sn(t|k^2) and t_j = i (j - 1/2) K'/N_p,
        A^{-1/2} ≈ (2 K' sqrt(m) / (pi N_p)) sum_{j=1}^{N_p} cn(t_j) dn(t_j) (A - w(t_j)^2 I)^{-1}.
    Readings taken here: the lower bound is m = min sigma^2 (the eigenvalues of A are at least
    the noise variance; the printed min sigma is not a bound in general) and the sum runs to N_p.
    For purely imaginary t = i u, Jacobi's imaginary transformation gives
        sn(iu|k^2) = i sc(u|1-k^2),  cn(iu|k^2) = 1/cn(u|1-k^2),  dn(iu|k^2) = dn(u|1-k^2)/cn(u|1-k^2),
    so the shifts are lambda_j = m sc^2(u_j|1-k^2) >= 0 and the weights are
        w_j = (2 K' sqrt(m) / (pi N_p)) dn(u_j|1-k^2) / cn(u_j|1-k^2)^2.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ellipj, ellipkm1
from scipy.linalg import cho_factor, cho_solve

from . import gp


def weights_shifts(m, M, n_poles=15):
    """(w_j, lambda_j), j = 1..n_poles, of the pole expansion of A^{-1/2} on [m, M]."""
    if not (0 < m <= M):
        raise ValueError("need 0 < m <= M")
    k2 = m / M
    kprime = ellipkm1(k2)                  # K(1 - k^2), accurate for small k^2
    u = (np.arange(1, n_poles + 1) - 0.5) * kprime / n_poles
    sn, cn, dn, _ = ellipj(u, 1.0 - k2)
    shifts = m * (sn / cn) ** 2
    weights = (2.0 * kprime * np.sqrt(m) / (np.pi * n_poles)) * dn / cn ** 2
    return weights, shifts


def gershgorin_upper(X, theta, kind):
    """Upper bound on lambda_max(A): the largest absolute row sum (all entries are positive)."""
    n = np.asarray(X).shape[0]
    return float(np.max(gp.matvec(X, theta, kind, np.ones(n))))


def inv_sqrt_apply(X, theta, kind, xi, n_poles=15, M=None):
    """phi ≈ A^{-1/2} xi by eq. (pex) with exact (Cholesky) shifted solves."""
    X = np.asarray(X, dtype=np.float64)
    A = gp.a_matrix(X, theta, kind)
    _, _, sigma2 = gp.unpack_theta(theta, kind, X.shape[1])
    if M is None:
        M = gershgorin_upper(X, theta, kind)
    w, lam = weights_shifts(sigma2, M, n_poles)
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros_like(xi)
    eye = np.eye(A.shape[0])
    for wp, lp in zip(w, lam):
        out += wp * cho_solve(cho_factor(A + lp * eye, lower=True), xi)
    return out
