"""Pins of the oracle's Chebyshev-amplitude kernel (Section 4):
K(x,x') = exp(C(x)) exp(C(x')) exp(-|x-x'|^2 / (2 l^2)), C(x) = sum_m Theta_m prod_k T_{m_k}(x^k).

Each pin is independent of the oracle's own arithmetic: the trigonometric definition of T_m,
a scalar math.exp loop, the reduction to the isotropic SE kernel when only Theta_0 is non-zero,
central finite differences of the dense quadratic form, and the row-partition identity.
"""
import math

import numpy as np
import pytest

from oracle import gp


def _theta(n_cheb, d, seed, ell=0.6, sigma2=0.1, scale=0.4):
    g = np.random.default_rng([seed, 77])
    return np.concatenate([scale * g.standard_normal(n_cheb ** d), [np.log(ell), np.log(sigma2)]])


def _points(n, d, seed):
    return np.random.default_rng([seed, 78]).uniform(-1.0, 1.0, size=(n, d))


def test_basis_matches_trigonometric_definition():
    # T_m(cos t) = cos(m t) on [-1, 1]; multi-index order m_1 slowest
    X = _points(7, 2, 1)
    B = gp.cheb_basis(X, 3)
    for i in range(7):
        for m1 in range(3):
            for m2 in range(3):
                ref = math.cos(m1 * math.acos(X[i, 0])) * math.cos(m2 * math.acos(X[i, 1]))
                assert abs(B[i, 3 * m1 + m2] - ref) < 1e-14


def test_kernel_entries_by_scalar_loop():
    n, d, nc = 5, 2, 3
    X = _points(n, d, 2)
    th = _theta(nc, d, 2)
    ell, s2 = math.exp(th[-2]), math.exp(th[-1])

    def C(x):
        s = 0.0
        for m1 in range(nc):
            for m2 in range(nc):
                s += th[nc * m1 + m2] * math.cos(m1 * math.acos(x[0])) * math.cos(m2 * math.acos(x[1]))
        return s

    A = gp.a_matrix(X, th, "cheb")
    for i in range(n):
        for j in range(n):
            r2 = sum((X[i, k] - X[j, k]) ** 2 for k in range(d))
            ref = math.exp(C(X[i])) * math.exp(C(X[j])) * math.exp(-r2 / (2 * ell * ell))
            if i == j:
                ref += s2
            assert abs(A[i, j] - ref) < 1e-13 * abs(ref)


def test_reduces_to_isotropic_se_with_constant_amplitude():
    # only Theta_0 = c non-zero: exp(C) = e^c, so K = e^{2c} K_SE, i.e. log alpha = 2c
    n, d, nc = 30, 2, 3
    X = _points(n, d, 3)
    c, ell, s2 = 0.37, 0.45, 0.05
    th = np.zeros(nc ** d + 2)
    th[0] = c
    th[-2:] = [np.log(ell), np.log(s2)]
    th_iso = np.array([2 * c, np.log(ell), np.log(s2)])
    np.testing.assert_allclose(gp.a_matrix(X, th, "cheb"), gp.a_matrix(X, th_iso, "iso"), rtol=1e-14)
    g = np.random.default_rng(4)
    U, V = g.standard_normal((n, 3)), g.standard_normal((n, 3))
    w = np.array([0.5, -1.0, 2.0])
    rc = gp.quadform_grad(X, th, "cheb", U, V, w)
    ri = gp.quadform_grad(X, th_iso, "iso", U, V, w)
    # dQ/dTheta_0 = dQ/dlog alpha * dlog alpha/dTheta_0 = 2 dQ/dlog alpha
    assert abs(rc["grad"][0] - 2 * ri["grad"][0]) < 1e-12 * abs(ri["grad"][0])
    assert abs(rc["grad"][-2] - ri["grad"][1]) < 1e-12 * abs(ri["grad"][1])
    assert abs(rc["grad"][-1] - ri["grad"][2]) < 1e-12 * abs(ri["grad"][2])
    np.testing.assert_allclose(rc["AU"], ri["AU"], rtol=1e-13)


@pytest.mark.parametrize("d,nc", [(1, 2), (2, 2), (1, 4), (3, 2)])
def test_gradient_by_central_differences(d, nc):
    n = 12
    X = _points(n, d, 10 + d + nc)
    th = _theta(nc, d, 5 + nc)
    g = np.random.default_rng([d, nc])
    U, V = g.standard_normal((n, 2)), g.standard_normal((n, 2))
    w = np.array([-0.5, 1.5])
    res = gp.quadform_grad(X, th, "cheb", U, V, w)
    h = 1e-5
    for p in range(len(th)):
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (gp.quadform_value(X, tp, "cheb", U, V, w) - gp.quadform_value(X, tm, "cheb", U, V, w)) / (2 * h)
        assert abs(res["grad"][p] - fd) < 1e-7 * (1 + abs(fd)), (p, res["grad"][p], fd)
    # q_c and the products by the dense matrix
    A = gp.a_matrix(X, th, "cheb")
    np.testing.assert_allclose(res["AU"], A @ U, rtol=1e-13)
    np.testing.assert_allclose(res["quad"], np.einsum("ic,ic->c", U, A @ V), rtol=1e-12)


def test_symmetric_positive_definite_and_row_partition():
    n, d, nc = 40, 2, 3
    X = _points(n, d, 6)
    th = _theta(nc, d, 6, sigma2=1e-3)
    A = gp.a_matrix(X, th, "cheb")
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A)[0] >= 1e-3 * (1 - 1e-9)
    g = np.random.default_rng(7)
    U = g.standard_normal((n, 2))
    full = gp.quadform_grad(X, th, "cheb", U, U)
    parts = [gp.quadform_grad(X, th, "cheb", U, U, rows=np.arange(s, min(n, s + 13))) for s in range(0, n, 13)]
    np.testing.assert_allclose(sum(p["grad"] for p in parts), full["grad"], rtol=1e-12)
    np.testing.assert_allclose(gp.matvec(X, th, "cheb", U), A @ U, rtol=1e-13)


def test_theta_length_checked():
    X = _points(4, 2, 8)
    with pytest.raises(ValueError):
        gp.a_matrix(X, np.zeros(7), "cheb")     # 5 is not N_cheb^2
    assert gp.n_theta("cheb", 3, 2) == 10
    assert gp.cheb_order(18, 2) == 4
