"""Oracle: exact hyperparameter posterior and the Gaussian-integral identity (FP64, CPU).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Definitions followed (paper section / equation):
  * P(theta) ∝ |A(theta)|^{-1/2} exp(-1/2 y^T A(theta)^{-1} y) p(theta)       (Section 2, eq. P)
    evaluated exactly with a Cholesky factor A = L L^T: log|A| = 2 sum_i log L_ii.
  * [det A]^{-1/2} ∝ integral over R^N of exp(-1/2 phi^T A phi) dphi; the constant is
    (2 pi)^{N/2} (Section 3, the pseudofermion identity).
  * The extended density P(theta, phi) ∝ exp(-[S + 1/2 y^T A^{-1} y + 1/2 phi^T A phi])
    (eq. extendeddensity), whose phi-marginal is P(theta).
  * Grid posterior on a box with the trapezoid rule (Section 4.1 uses a 100^2 grid on [-3,3]^2).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from . import gp


def log_posterior(X, theta, kind, y, prior=None):
    """log P(theta) up to its normalising constant (eq. P), by Cholesky."""
    A = gp.a_matrix(X, theta, kind)
    c, low = cho_factor(A, lower=True)
    y = np.asarray(y, dtype=np.float64)
    x = cho_solve((c, low), y)
    logdet = 2.0 * np.sum(np.log(np.diag(c)))
    s = 0.0 if prior is None else float(prior(theta))
    return -0.5 * logdet - 0.5 * float(y @ x) - s


def grid_log_posterior(X, kind, y, theta_base, idx, axes, prior=None):
    """log P on the tensor grid axes[0] x axes[1] for the components idx of theta."""
    out = np.empty((len(axes[0]), len(axes[1])))
    th = np.array(theta_base, dtype=np.float64)
    for a, va in enumerate(axes[0]):
        for b, vb in enumerate(axes[1]):
            th[idx[0]] = va
            th[idx[1]] = vb
            out[a, b] = log_posterior(X, th, kind, y, prior)
    return out


def trapezoid_weights(x):
    """Composite trapezoid weights for the ordered nodes x."""
    x = np.asarray(x, dtype=np.float64)
    w = np.zeros_like(x)
    dx = np.diff(x)
    w[:-1] += 0.5 * dx
    w[1:] += 0.5 * dx
    return w


def grid_marginals(logp, axes):
    """Normalised marginal densities and CDFs of a 2-D grid log density (trapezoid rule)."""
    p = np.exp(logp - logp.max())
    w0 = trapezoid_weights(axes[0])
    w1 = trapezoid_weights(axes[1])
    z = w0 @ p @ w1
    m0 = (p @ w1) / z
    m1 = (w0 @ p) / z
    cdfs = []
    for m, ax in ((m0, axes[0]), (m1, axes[1])):
        c = np.concatenate([[0.0], np.cumsum(0.5 * (m[1:] + m[:-1]) * np.diff(ax))])
        cdfs.append(c)
    return (m0, m1), tuple(cdfs)


def gaussian_integral(A, n_nodes=121, half_width=None):
    """(2 pi)^{-N/2} * integral of exp(-1/2 z^T A z) over R^N by the tensor trapezoid rule.

    For N <= 3 only.  The integrand is a Gaussian, so the trapezoid rule on a box of half width
    12/sqrt(lambda_min) is spectrally accurate; the exact value is det(A)^{-1/2}.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if n > 3:
        raise ValueError("tensor quadrature only for N <= 3")
    if half_width is None:
        half_width = 12.0 / np.sqrt(np.linalg.eigvalsh(A).min())
    t = np.linspace(-half_width, half_width, n_nodes)
    w = trapezoid_weights(t)
    grids = np.meshgrid(*([t] * n), indexing="ij")
    Z = np.stack([g.ravel() for g in grids], axis=1)
    W = np.ones(Z.shape[0])
    Wg = np.meshgrid(*([w] * n), indexing="ij")
    for g in Wg:
        W = W * g.ravel()
    q = np.einsum("pi,ij,pj->p", Z, A, Z)
    total = float(np.sum(W * np.exp(-0.5 * q)))
    return total / (2.0 * np.pi) ** (n / 2.0)


def log_phi_marginal(X, theta, kind, y, n_nodes=121, prior=None):
    """log of the integral over phi of exp(-[S + 1/2 y^T A^{-1} y + 1/2 phi^T A phi]).

    By the pseudofermion identity this equals log P(theta) + (N/2) log(2 pi) (for N <= 3).
    """
    A = gp.a_matrix(X, theta, kind)
    y = np.asarray(y, dtype=np.float64)
    x = cho_solve(cho_factor(A, lower=True), y)
    s = 0.0 if prior is None else float(prior(theta))
    gi = gaussian_integral(A, n_nodes) * (2.0 * np.pi) ** (A.shape[0] / 2.0)
    return np.log(gi) - 0.5 * float(y @ x) - s
