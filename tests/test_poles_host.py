"""Host side of the Gibbs refresh of phi: the pole weights and shifts of Appendix A (eq. msqdisc)
computed by the library (host code, no GPU), pinned against 50-digit mpmath values and against
the oracle; argument checks of gp_phi_refresh before any HIP call; workspace sizing."""
import ctypes
import os

import mpmath
import numpy as np
import pytest

from oracle import poles as opoles
from paper_2412_20884_amd import gpk

pytestmark = pytest.mark.skipif(not os.path.exists(gpk.LIB_PATH), reason="libgpk.so not built")


def mp_weights_shifts(m, M, n_poles, dps=50):
    """Weights and shifts at `dps` digits, straight from the imaginary-node form of eq. (msqdisc):
    t_j = i (j - 1/2) K' / N_p, w(t) = sqrt(m) sn(t | k^2), weight 2 K' sqrt(m) / (pi N_p) cn dn,
    term (A - w^2 I)^{-1}, i.e. shift -w^2 -- evaluated with complex Jacobi functions, so the
    imaginary transformation the library relies on is not used here."""
    with mpmath.workdps(dps):
        m_, M_ = mpmath.mpf(m), mpmath.mpf(M)
        k2 = m_ / M_
        kp = mpmath.ellipk(1 - k2)
        ws, ss = [], []
        for j in range(1, n_poles + 1):
            t = mpmath.mpc(0, (j - mpmath.mpf(1) / 2) * kp / n_poles)
            sn = mpmath.ellipfun("sn", t, m=k2)
            cn = mpmath.ellipfun("cn", t, m=k2)
            dn = mpmath.ellipfun("dn", t, m=k2)
            wt = mpmath.sqrt(m_) * sn
            weight = 2 * kp * mpmath.sqrt(m_) / (mpmath.pi * n_poles) * cn * dn
            shift = -(wt ** 2)
            assert abs(mpmath.im(weight)) < mpmath.mpf(10) ** (-dps // 2) * abs(weight)
            assert abs(mpmath.im(shift)) < mpmath.mpf(10) ** (-dps // 2) * (1 + abs(shift))
            ws.append(float(mpmath.re(weight)))
            ss.append(float(mpmath.re(shift)))
    return np.array(ws), np.array(ss)


@pytest.mark.parametrize("m,M,n_poles", [(1e-2, 76.9, 15), (0.3, 0.3, 4), (1.0, 3.0, 1),
                                         (1e-4, 1e4, 15), (1e-6, 1e6, 40), (2e-3, 1.0, 7)])
def test_pole_weights_vs_mpmath(m, M, n_poles):
    w, s = gpk.pole_weights(m, M, n_poles)
    wr, sr = mp_weights_shifts(m, M, n_poles)
    assert np.all(s >= 0) and np.all(np.diff(s) > 0) or n_poles == 1
    # near u = K'/2, cn ~ sqrt(k): at m / M = 1e-12 the middle nodes keep ~11 digits, still far
    # below the expansion's own error there
    tol = 1e-12 if m / M >= 1e-9 else 1e-10
    assert np.max(np.abs(w - wr) / np.abs(wr)) < tol
    assert np.max(np.abs(s - sr) / np.maximum(np.abs(sr), 1e-300)) < tol


@pytest.mark.parametrize("m,M,n_poles", [(1e-2, 76.9, 15), (1e-3, 10.0, 10), (0.05, 2.0, 20)])
def test_pole_weights_vs_oracle(m, M, n_poles):
    # the oracle passes the parameter 1 - k^2 to SciPy, which loses relative accuracy in k^2
    # as m / M -> 0; at these ratios both agree far below the expansion's own error
    w, s = gpk.pole_weights(m, M, n_poles)
    wo, so = opoles.weights_shifts(m, M, n_poles)
    assert np.max(np.abs(w - wo) / np.abs(wo)) < 1e-10
    assert np.max(np.abs(s - so) / so) < 1e-10


def test_pole_weights_scalar_case():
    # on a one-point spectrum [m, m] (k = 1) the nodes are circular, lambda_j = m tan^2 u_j and
    # w_j = sqrt(m) / (N_p cos^2 u_j), so sum_j w_j / (m + lambda_j) = m^{-1/2} for every N_p
    for n_poles in (1, 3, 15):
        w, s = gpk.pole_weights(0.7, 0.7, n_poles)
        val = np.sum(w / (0.7 + s))
        assert abs(val - 0.7 ** -0.5) < 1e-13 * 0.7 ** -0.5


def test_pole_weights_rejects_bad_arguments():
    L = gpk.lib()
    buf = (ctypes.c_double * 4)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.gp_pole_weights(0.0, 1.0, 4, p, p) == 1
    assert L.gp_pole_weights(2.0, 1.0, 4, p, p) == 1
    assert L.gp_pole_weights(1.0, float("inf"), 4, p, p) == 1
    assert L.gp_pole_weights(0.1, 1.0, 0, p, p) == 1
    assert L.gp_pole_weights(0.1, 1.0, 4, None, p) == 1


def _phi(k, prm, n=10, X=1, th=1, r=2, xi=4096, ldxi=2, phi=1 << 20, ldphi=2, ws=8, wsb=1 << 40):
    L = gpk.lib()
    vp = ctypes.c_void_p
    return L.gp_phi_refresh(k, prm, n, vp(X), vp(th), r, vp(xi), ldxi, vp(phi), ldphi, None, None,
                            None, vp(ws), wsb, None)


def test_phi_refresh_validation():
    good = ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 3, 0))
    prm = gpk.PhiParams(15, 1e-8, 100, 0.0)
    P = ctypes.byref(prm)
    assert _phi(None, P) == 1
    assert _phi(good, None) == 1
    assert _phi(ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 3, gpk.NO_NOISE)), P) == 1
    assert _phi(good, P, r=0) == 2
    assert _phi(good, P, r=33) == 2
    assert _phi(good, P, n=-1) == 2
    for bad in (gpk.PhiParams(0, 1e-8, 100, 0.0), gpk.PhiParams(65, 1e-8, 100, 0.0),
                gpk.PhiParams(15, 0.0, 100, 0.0), gpk.PhiParams(15, 1e-8, 0, 0.0),
                gpk.PhiParams(15, 1e-8, 10, float("inf"))):
        assert _phi(good, ctypes.byref(bad)) == 1
    assert _phi(good, P, X=0) == 1
    assert _phi(good, P, ldxi=1) == 2
    assert _phi(good, P, ldphi=1) == 2
    assert _phi(good, P, xi=4096, phi=4100) == 1        # partial overlap
    assert _phi(good, P, ws=0) == 4
    assert _phi(good, P, wsb=64) == 4


def test_phi_workspace_size():
    L = gpk.lib()
    k = ctypes.byref(gpk.Kernel(gpk.ARD, gpk.F32, 8, 0))
    p15 = gpk.PhiParams(15, 1e-8, 100, 0.0)
    p30 = gpk.PhiParams(30, 1e-8, 100, 0.0)
    a = L.gp_phi_workspace_size(k, ctypes.byref(p15), 1000, 1)
    b = L.gp_phi_workspace_size(k, ctypes.byref(p15), 1000, 4)
    c = L.gp_phi_workspace_size(k, ctypes.byref(p30), 1000, 4)
    d = L.gp_phi_workspace_size(k, ctypes.byref(p15), 100000, 4)
    assert 0 < a < b < c and b < d
    # the shifted directions dominate: at least n_poles * n * r floats
    assert d >= 15 * 100000 * 4 * 4
    assert L.gp_phi_workspace_size(k, ctypes.byref(p15), 0, 4) == 0
    assert L.gp_phi_workspace_size(k, ctypes.byref(gpk.PhiParams(0, 1e-8, 100, 0.0)), 10, 1) == 0
