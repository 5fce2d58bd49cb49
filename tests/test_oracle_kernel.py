"""Pins of the oracle's kernel matrix, matvec and quadratic-form gradient.

Each test checks the oracle against something other than itself: a closed form, a limit,
an invariant, a brute-force scalar loop, or central finite differences of a different code path.
"""
import math

import numpy as np
import pytest

from oracle import gp
from paper_2412_20884_amd import inputs as I


def brute_A(X, theta, kind):
    """Scalar double loop with math.exp: A_ij = sigma^2 delta_ij + alpha exp(-1/2 sum (dx/l)^2)."""
    n, d = len(X), len(X[0])
    a = math.exp(theta[0])
    ells = [math.exp(theta[1])] * d if kind == "iso" else [math.exp(t) for t in theta[1:1 + d]]
    s2 = math.exp(theta[-1])
    A = [[0.0] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            e = 0.0
            for k in range(d):
                e += ((X[i][k] - X[j][k]) / ells[k]) ** 2
            A[i][j] = a * math.exp(-0.5 * e) + (s2 if i == j else 0.0)
    return np.array(A)


def test_closed_form_two_points_iso():
    # Section 1 SE kernel at N=2, d=1: A = [[a+s2, a e^{-r^2/(2 l^2)}], [., a+s2]]
    X = np.array([[0.3], [0.75]])
    alpha, ell, s2 = 1.7, 0.4, 0.05
    th = np.log([alpha, ell, s2])
    A = gp.a_matrix(X, th, "iso")
    off = alpha * math.exp(-(0.45 ** 2) / (2 * ell ** 2))
    np.testing.assert_allclose(A, [[alpha + s2, off], [off, alpha + s2]], rtol=1e-15)


def test_closed_form_two_points_ard():
    X = np.array([[0.1, -0.2], [0.4, 0.5]])
    alpha, l1, l2, s2 = 0.8, 0.5, 2.0, 0.01
    th = np.log([alpha, l1, l2, s2])
    A = gp.a_matrix(X, th, "ard")
    off = alpha * math.exp(-0.5 * ((0.3 / l1) ** 2 + (0.7 / l2) ** 2))
    np.testing.assert_allclose(A, [[alpha + s2, off], [off, alpha + s2]], rtol=1e-15)


def test_limits():
    X = I.uniform_points(9, 2, 7)
    # very long length-scale: K -> alpha 1 1^T
    A = gp.a_matrix(X, np.log([2.0, 1e6, 0.1]), "iso")
    np.testing.assert_allclose(A, 2.0 * np.ones((9, 9)) + 0.1 * np.eye(9), rtol=1e-10)
    # points far apart relative to l: A -> (alpha + s2) I
    Xf = np.arange(5.0)[:, None] * 100.0
    A = gp.a_matrix(Xf, np.log([2.0, 1.0, 0.1]), "iso")
    np.testing.assert_allclose(A, 2.1 * np.eye(5), atol=1e-300)
    # no_noise gives the kernel matrix of eq. (kernmat)
    K = gp.a_matrix(X, np.log([2.0, 0.3, 0.1]), "iso", no_noise=True)
    np.testing.assert_allclose(np.diag(K), 2.0, rtol=1e-15)


@pytest.mark.parametrize("kind,d", [("iso", 1), ("iso", 3), ("ard", 3), ("ard", 5)])
def test_brute_force_and_invariants(kind, d):
    g = np.random.default_rng(11 + d)
    X = g.normal(size=(7, d))
    th = np.concatenate([[0.3], g.uniform(-1, 0.5, size=1 if kind == "iso" else d), [np.log(0.02)]])
    A = gp.a_matrix(X, th, kind)
    np.testing.assert_allclose(A, brute_A(X.tolist(), th, kind), rtol=1e-14, atol=1e-300)
    np.testing.assert_array_equal(A, A.T)
    lam = np.linalg.eigvalsh(A)
    assert lam.min() >= 0.02 - 1e-12
    np.linalg.cholesky(A)


@pytest.mark.parametrize("kind,d", [("iso", 2), ("ard", 4)])
def test_matvec_blocked_vs_dense(kind, d, monkeypatch):
    g = np.random.default_rng(5)
    n = 37
    X = g.normal(size=(n, d))
    th = np.concatenate([[0.1], g.uniform(-0.5, 0.5, size=1 if kind == "iso" else d), [-3.0]])
    V = g.normal(size=(n, 3))
    shift = np.array([0.0, 0.5, 2.0])
    ref = np.stack([(brute_A(X.tolist(), th, kind) + s * np.eye(n)) @ V[:, c] for c, s in enumerate(shift)], 1)
    # force many small row blocks so the partition is exercised
    monkeypatch.setattr(gp, "_row_blocks", lambda rows, n_cols, max_entries=0: [rows[i:i + 5] for i in range(0, len(rows), 5)])
    out = gp.matvec(X, th, kind, V, col_shift=shift)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)
    rows = np.array([3, 17, 36])
    np.testing.assert_allclose(gp.matvec(X, th, kind, V, col_shift=shift, rows=rows), ref[rows], rtol=1e-13)
    # symmetric operator: u^T (A v) = v^T (A u); z^T A z >= sigma^2 |z|^2
    u, v = V[:, 0], V[:, 1]
    assert abs(u @ gp.matvec(X, th, kind, v) - v @ gp.matvec(X, th, kind, u)) < 1e-12
    assert v @ gp.matvec(X, th, kind, v) >= math.exp(-3.0) * (v @ v)


def test_gradient_two_point_closed_form():
    # N=2, d=1: dQ/dlog a = a(u.v) + a e (u1 v2 + u2 v1); dQ/dlog l = a e (r^2/l^2)(u1 v2 + u2 v1);
    # dQ/dlog s2 = s2 (u.v), with e = exp(-r^2/(2 l^2))
    X = np.array([[0.0], [0.6]])
    a, l, s2 = 1.3, 0.5, 0.07
    u = np.array([0.7, -1.1])
    v = np.array([0.4, 2.0])
    r2 = 0.36
    e = math.exp(-r2 / (2 * l * l))
    cross = u[0] * v[1] + u[1] * v[0]
    expect = [a * (u @ v) + a * e * cross, a * e * (r2 / l ** 2) * cross, s2 * (u @ v)]
    res = gp.quadform_grad(X, np.log([a, l, s2]), "iso", u, v)
    np.testing.assert_allclose(res["grad"], expect, rtol=1e-14)
    A = np.array([[a + s2, a * e], [a * e, a + s2]])
    np.testing.assert_allclose(res["quad"], [u @ A @ v], rtol=1e-14)


@pytest.mark.parametrize("kind,d", [("iso", 2), ("iso", 3), ("ard", 3), ("ard", 6)])
def test_gradient_central_fd(kind, d):
    g = np.random.default_rng(100 + d)
    n, R = 23, 3
    X = g.normal(size=(n, d)) * 0.7
    th = np.concatenate([[0.2], g.uniform(-0.6, 0.3, size=1 if kind == "iso" else d), [np.log(0.05)]])
    U = g.normal(size=(n, R))
    V = g.normal(size=(n, R))
    w = np.array([0.5, -1.25, 2.0])
    res = gp.quadform_grad(X, th, kind, U, V, w)
    h = 1e-5
    fd = np.zeros_like(th)
    for p in range(len(th)):
        e = np.zeros_like(th)
        e[p] = h
        fd[p] = (gp.quadform_value(X, th + e, kind, U, V, w) - gp.quadform_value(X, th - e, kind, U, V, w)) / (2 * h)
    scale = np.abs(res["grad"]).max()
    np.testing.assert_allclose(res["grad"], fd, rtol=1e-7, atol=1e-8 * scale)
    A = gp.a_matrix(X, th, kind)
    np.testing.assert_allclose(res["AU"], A @ U, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(res["AV"], A @ V, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(res["quad"], np.einsum("ic,ij,jc->c", U, A, V), rtol=1e-12)


def test_row_partition_sums_to_full():
    p = I.ard_problem(40, 3, 9)
    full = gp.quadform_grad(p["X"], p["theta"], "ard", p["U"], p["V"])
    a = gp.quadform_grad(p["X"], p["theta"], "ard", p["U"], p["V"], rows=np.arange(0, 17))
    b = gp.quadform_grad(p["X"], p["theta"], "ard", p["U"], p["V"], rows=np.arange(17, 40))
    np.testing.assert_allclose(a["grad"] + b["grad"], full["grad"], rtol=1e-12)
    np.testing.assert_allclose(a["quad"] + b["quad"], full["quad"], rtol=1e-12)
    np.testing.assert_allclose(np.vstack([a["AV"], b["AV"]]), full["AV"], rtol=1e-14)


def test_ard_identity_reduces_to_iso():
    # ARD with all length-scales equal is the isotropic kernel; the iso l-gradient is the sum
    # of the ARD per-coordinate gradients.
    p = I.iso_problem(30, 3, 4)
    th_iso = p["theta"]
    th_ard = np.concatenate([[th_iso[0]], [th_iso[1]] * 3, [th_iso[2]]])
    gi = gp.quadform_grad(p["X"], th_iso, "iso", p["U"], p["V"])
    ga = gp.quadform_grad(p["X"], th_ard, "ard", p["U"], p["V"])
    np.testing.assert_allclose(ga["AV"], gi["AV"], rtol=1e-14)
    np.testing.assert_allclose(ga["grad"][1:4].sum(), gi["grad"][1], rtol=1e-12)
    np.testing.assert_allclose(ga["grad"][[0, 4]], gi["grad"][[0, 2]], rtol=1e-13)


def test_row_restricted_gradient_brute_force():
    # With rows given, the i index of u_ic runs over those rows only:
    # g_p = sum_{i in rows} sum_j sum_c w_c u_ic v_jc dA_ij/dtheta_p, checked with scalar loops.
    p = I.ard_problem(9, 2, 12)
    X, th = p["X"], p["theta"]
    U, V = p["U"][:, :2], p["V"][:, :2]
    w = np.array([0.7, -1.3])
    rows = [1, 4, 8]
    a = math.exp(th[0])
    ells = [math.exp(t) for t in th[1:3]]
    s2 = math.exp(th[-1])
    g = np.zeros(4)
    for i in rows:
        for j in range(9):
            dk = [((X[i, k] - X[j, k]) / ells[k]) ** 2 for k in range(2)]
            kij = a * math.exp(-0.5 * sum(dk))
            s = sum(w[c] * U[i, c] * V[j, c] for c in range(2))
            g[0] += kij * s
            g[1] += kij * dk[0] * s
            g[2] += kij * dk[1] * s
            if i == j:
                g[3] += s2 * s
    res = gp.quadform_grad(X, th, "ard", U, V, w, rows=np.array(rows))
    np.testing.assert_allclose(res["grad"], g, rtol=1e-13)
