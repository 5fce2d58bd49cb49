"""Oracle: chain statistics used by the statistical tests (CPU).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

  * Integrated autocorrelation time, Appendix C: C_hat(j) = 1/(N-j) sum (f_i - mean)(f_{i+j} - mean),
    tau_hat = 1 + 2 sum_{j=1}^{M} C_hat(j)/C_hat(0) with the window M the smallest value
    satisfying M >= c tau_hat (c = 5).  For B independent chains of one target (Section 4.1
    runs B = 500) the same estimator is applied to C_hat(j) averaged over the chains, each chain
    centred on the mean of all chains.
  * Moving-window mean T_i = mean(X_{floor(i/2)}, ..., X_i), Section 4.1.
  * Dvoretzky-Kiefer-Wolfowitz radius of an empirical CDF with n effective samples:
    sqrt(log(2/delta) / (2 n)).
"""
from __future__ import annotations

import numpy as np


def autocov(f):
    f = np.asarray(f, dtype=np.float64)
    n = len(f)
    g = f - f.mean()
    return np.array([np.dot(g[: n - j], g[j:]) / (n - j) for j in range(n)])


def _tau_from_autocov(C, c):
    if C[0] <= 0:
        return 1.0
    rho = C / C[0]
    tau = 1.0
    for m in range(1, len(C)):
        tau = 1.0 + 2.0 * np.sum(rho[1:m + 1])
        if m >= c * tau:
            return float(tau)
    return float(tau)


def iat(f, c=5.0):
    """tau_hat with the automatic window M >= c tau_hat (Appendix C)."""
    return _tau_from_autocov(autocov(f), c)


def iat_chains(F, c=5.0, max_lag=None):
    """tau_hat of B chains (rows of F, equal lengths L) from the chain-averaged autocovariance
    C_hat(j) = 1/(B (L-j)) sum_b sum_i (f_bi - mean)(f_b,i+j - mean), mean over all chains;
    window as in iat.  max_lag bounds the lags evaluated (default L - 1)."""
    F = np.asarray(F, dtype=np.float64)
    if F.ndim == 1:
        F = F[None, :]
    B, L = F.shape
    G = F - F.mean()
    top = L if max_lag is None else min(L, int(max_lag) + 1)
    C = np.array([np.sum(G[:, : L - j] * G[:, j:]) / (B * (L - j)) for j in range(top)])
    return _tau_from_autocov(C, c)


def moving_window_mean(x):
    x = np.asarray(x, dtype=np.float64)
    cs = np.concatenate([[0.0], np.cumsum(x)])
    i = np.arange(len(x))
    lo = i // 2
    return (cs[i + 1] - cs[lo]) / (i + 1 - lo)


def dkw_radius(n_eff, delta=0.05):
    return float(np.sqrt(np.log(2.0 / delta) / (2.0 * n_eff)))
