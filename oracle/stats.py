"""Oracle: chain statistics used by the statistical tests (CPU).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

  * Integrated autocorrelation time, Appendix C: C_hat(j) = 1/(N-j) sum (f_i - mean)(f_{i+j} - mean),
    tau_hat = 1 + 2 sum_{j=1}^{M} C_hat(j)/C_hat(0) with the window M the smallest value
    satisfying M >= c tau_hat (c = 5).
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


def iat(f, c=5.0):
    """tau_hat with the automatic window M >= c tau_hat (Appendix C)."""
    C = autocov(f)
    if C[0] <= 0:
        return 1.0
    rho = C / C[0]
    tau = 1.0
    for m in range(1, len(f)):
        tau = 1.0 + 2.0 * np.sum(rho[1:m + 1])
        if m >= c * tau:
            return float(tau)
    return float(tau)


def moving_window_mean(x):
    x = np.asarray(x, dtype=np.float64)
    cs = np.concatenate([[0.0], np.cumsum(x)])
    i = np.arange(len(x))
    lo = i // 2
    return (cs[i + 1] - cs[lo]) / (i + 1 - lo)


def dkw_radius(n_eff, delta=0.05):
    return float(np.sqrt(np.log(2.0 / delta) / (2.0 * n_eff)))
