"""Pins of the pole expansion (Appendix A) and the chain statistics (Appendix C)."""
import numpy as np
import pytest

from oracle import gp, poles, stats
from paper_2412_20884_amd import inputs as I


def _inv_sqrt_eigh(A, xi):
    lam, Q = np.linalg.eigh(A)
    return Q @ ((Q.T @ xi) / np.sqrt(lam))


def test_pole_expansion_converges_to_eigh():
    p = I.iso_problem(150, 2, 21, ell=0.2, sigma2=1e-2)
    A = gp.a_matrix(p["X"], p["theta"], "iso")
    ref = _inv_sqrt_eigh(A, p["xi"])
    errs = []
    for npole in (5, 10, 15):
        phi = poles.inv_sqrt_apply(p["X"], p["theta"], "iso", p["xi"], n_poles=npole)
        errs.append(np.linalg.norm(phi - ref) / np.linalg.norm(ref))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-9, errs


def test_pole_expansion_scalar_bound():
    # On scalars a in [m, M] the expansion approximates a^{-1/2} with error decaying like
    # exp(-2 pi K N_p / K'), Appendix A.
    from scipy.special import ellipk, ellipkm1
    m, M = 1e-2, 50.0
    a = np.geomspace(m, M, 200)
    for npole in (6, 12):
        w, lam = poles.weights_shifts(m, M, npole)
        approx = np.sum(w[None, :] / (a[:, None] + lam[None, :]), axis=1)
        err = np.max(np.abs(approx * np.sqrt(a) - 1.0))
        K, Kp = ellipk(m / M), ellipkm1(m / M)
        assert err < 50 * np.exp(-2 * np.pi * K * npole / Kp), (npole, err)
    assert np.all(lam >= 0)


def test_gershgorin_bounds_spectrum():
    p = I.iso_problem(60, 2, 3, ell=0.3)
    A = gp.a_matrix(p["X"], p["theta"], "iso")
    assert poles.gershgorin_upper(p["X"], p["theta"], "iso") >= np.linalg.eigvalsh(A).max()


def test_iat_ar1():
    # AR(1) with coefficient r has tau = (1 + r)/(1 - r)
    g = np.random.default_rng(0)
    r = 0.8
    n = 100000
    x = np.empty(n)
    x[0] = g.normal()
    e = g.normal(size=n) * np.sqrt(1 - r * r)
    for t in range(1, n):
        x[t] = r * x[t - 1] + e[t]
    tau = stats.iat(x[:20000])
    assert abs(tau - 9.0) < 1.5


def test_moving_window_mean():
    x = np.arange(10.0)
    T = stats.moving_window_mean(x)
    for i in range(10):
        assert T[i] == pytest.approx(np.mean(x[i // 2:i + 1]))
