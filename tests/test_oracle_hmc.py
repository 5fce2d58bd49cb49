"""Pins of the oracle's solve, potential, force, leapfrog and Hamiltonian.

The force is pinned to central finite differences of the exact-solve potential (which pins the
frozen-x evaluation and its sign); the integrator to reversibility, second order and volume
preservation; the identity behind the auxiliary variable to quadrature.
"""
import math

import numpy as np
import pytest

from oracle import gp, hmc, posterior
from paper_2412_20884_amd import inputs as I


def _problem(n=24, d=2, seed=3, kind="iso"):
    if kind == "iso":
        p = I.iso_problem(n, d, seed, ell=0.35, sigma2=0.05)
    else:
        p = I.ard_problem(n, d, seed, sigma2=0.05)
    X, y, th = p["X"], p["y"], p["theta"]
    phi = np.random.default_rng(seed).normal(size=n) * 0.5
    return X, y, th, phi


def test_solve_residual():
    X, y, th, _ = _problem()
    x = hmc.solve(X, th, "iso", y)
    np.testing.assert_allclose(gp.a_matrix(X, th, "iso") @ x, y, atol=1e-11)


@pytest.mark.parametrize("kind,d", [("iso", 2), ("ard", 3)])
def test_force_is_gradient_of_potential(kind, d):
    X, y, th, phi = _problem(d=d, kind=kind)
    F = hmc.force(X, th, kind, y, phi)
    h = 1e-5
    for p in range(len(th)):
        e = np.zeros_like(th)
        e[p] = h
        fd = (hmc.potential(X, th + e, kind, y, phi) - hmc.potential(X, th - e, kind, y, phi)) / (2 * h)
        assert abs(F[p] - fd) <= 1e-7 * max(1.0, abs(fd)), (p, F[p], fd)


def test_variational_energy_form():
    X, y, th, phi = _problem()
    x = hmc.solve(X, th, "iso", y)
    U = hmc.potential(X, th, "iso", y, phi)
    assert abs(hmc.potential_at(X, th, "iso", y, phi, x) - U) < 1e-10 * abs(U)
    # second order in the residual: perturb x by eps -> error ~ eps^2
    g = np.random.default_rng(0).normal(size=len(y))
    e1 = hmc.potential_at(X, th, "iso", y, phi, x + 1e-3 * g) - U
    e2 = hmc.potential_at(X, th, "iso", y, phi, x + 2e-3 * g) - U
    assert e1 < 0 and e2 < 0 and 3.5 < e2 / e1 < 4.5


def test_leapfrog_reversible():
    X, y, th, phi = _problem()
    pi0 = np.array([0.3, -0.7, 0.2])
    th1, pi1 = hmc.leapfrog(X, "iso", y, phi, th, pi0, 0.05, 6)
    th2, pi2 = hmc.leapfrog(X, "iso", y, phi, th1, -pi1, 0.05, 6)
    np.testing.assert_allclose(th2, th, atol=1e-11)
    np.testing.assert_allclose(-pi2, pi0, atol=1e-11)


def test_leapfrog_second_order_energy_error():
    X, y, th, phi = _problem()
    pi0 = np.array([0.5, -0.4, 0.3])
    T = 0.4
    errs = []
    for n in (4, 8, 16):
        th1, pi1 = hmc.leapfrog(X, "iso", y, phi, th, pi0, T / n, n)
        errs.append(abs(hmc.hamiltonian(X, th1, "iso", y, phi, pi1) - hmc.hamiltonian(X, th, "iso", y, phi, pi0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs


def test_leapfrog_one_step_matches_definition():
    # one DKD step written out: theta_1/2 = theta + dt/2 pi; pi' = pi - dt F(theta_1/2);
    # theta' = theta_1/2 + dt/2 pi'.  The force is taken from finite differences of U so this
    # does not reuse the oracle's force routine.
    X, y, th, phi = _problem()
    pi0 = np.array([0.2, 0.1, -0.3])
    dt = 0.1
    th_h = th + 0.5 * dt * pi0
    h = 1e-6
    F = np.array([(hmc.potential(X, th_h + h * e, "iso", y, phi) - hmc.potential(X, th_h - h * e, "iso", y, phi)) / (2 * h)
                  for e in np.eye(3)])
    pi1 = pi0 - dt * F
    th1 = th_h + 0.5 * dt * pi1
    a, b = hmc.leapfrog(X, "iso", y, phi, th, pi0, dt, 1)
    np.testing.assert_allclose(a, th1, atol=1e-8)
    np.testing.assert_allclose(b, pi1, atol=1e-8)


def test_leapfrog_volume_preserving():
    X, y, th, phi = _problem(n=12)
    z0 = np.concatenate([th, [0.2, -0.1, 0.4]])

    def flow(z):
        a, b = hmc.leapfrog(X, "iso", y, phi, z[:3], z[3:], 0.1, 3)
        return np.concatenate([a, b])

    h = 1e-6
    J = np.stack([(flow(z0 + h * e) - flow(z0 - h * e)) / (2 * h) for e in np.eye(6)], axis=1)
    assert abs(np.linalg.det(J) - 1.0) < 1e-6


def test_accept_rule():
    assert hmc.accept(5.0, 5.0, 0.999)
    assert hmc.accept(5.0, 6.0, math.exp(-1.0) - 1e-12)
    assert not hmc.accept(5.0, 6.0, math.exp(-1.0) + 1e-9)
    assert hmc.accept(0.0, 100.0, 0.0)


def test_trajectory_reject_restores():
    # A downhill trajectory run backwards from its end point with the momentum negated is
    # uphill by the same energy change (reversibility), so both Metropolis branches are reached.
    X, y, th, phi = _problem()
    fwd = hmc.trajectory(X, "iso", y, phi, th, np.array([3.0, 3.0, 3.0]), 0.3, 5)
    assert fwd["H1"] < fwd["H0"] - 0.1
    th1, pi1 = fwd["theta_prop"], -fwd["pi_prop"]
    p_acc = math.exp(fwd["H1"] - fwd["H0"])  # acceptance probability of the uphill move
    rej = hmc.trajectory(X, "iso", y, phi, th1, pi1, 0.3, 5, u=min(1.0, p_acc + 0.2))
    assert rej["H1"] - rej["H0"] == pytest.approx(fwd["H0"] - fwd["H1"], abs=1e-9)
    assert not rej["accepted"]
    np.testing.assert_array_equal(rej["theta"], th1)
    np.testing.assert_array_equal(rej["pi"], pi1)
    np.testing.assert_allclose(rej["theta_prop"], th, atol=1e-10)
    acc = hmc.trajectory(X, "iso", y, phi, th1, pi1, 0.3, 5, u=p_acc - 0.2)
    assert acc["accepted"]
    np.testing.assert_allclose(acc["theta"], th, atol=1e-10)
    np.testing.assert_array_equal(acc["theta"], acc["theta_prop"])


def test_inverse_mass_identity_and_frozen_component():
    X, y, th, phi = _problem()
    pi0 = np.array([0.7, -0.4, 0.9])
    a = hmc.leapfrog(X, "iso", y, phi, th, pi0, 0.05, 4)
    b = hmc.leapfrog(X, "iso", y, phi, th, pi0, 0.05, 4, inv_mass=np.ones(3))
    np.testing.assert_array_equal(a[0], b[0])
    # a zero inverse mass holds that component fixed and removes its kinetic energy
    minv = np.array([1.0, 0.5, 0.0])
    th1, pi1 = hmc.leapfrog(X, "iso", y, phi, th, pi0, 0.05, 4, inv_mass=minv)
    assert th1[2] == th[2] and th1[0] != th[0] and th1[1] != th[1]
    H = hmc.hamiltonian(X, th, "iso", y, phi, pi0, inv_mass=minv)
    assert H == pytest.approx(hmc.potential(X, th, "iso", y, phi) + 0.5 * (0.49 + 0.5 * 0.16), abs=1e-12)
    # with the third component frozen the flow is the M = diag(1, 2) flow of the first two with
    # sigma^2 fixed: energy error second order in the step, reversible
    errs = []
    for dt, ns in ((0.04, 5), (0.02, 10)):
        t1, p1 = hmc.leapfrog(X, "iso", y, phi, th, pi0, dt, ns, inv_mass=minv)
        errs.append(abs(hmc.hamiltonian(X, t1, "iso", y, phi, p1, inv_mass=minv) - H))
        tb, pb = hmc.leapfrog(X, "iso", y, phi, t1, -p1, dt, ns, inv_mass=minv)
        np.testing.assert_allclose(tb, th, atol=1e-11)
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_rwm_inverse_mass_scales_step():
    X, y, th, phi = _problem()
    xi = np.array([0.3, -0.2, 0.5])
    r = hmc.rwm_update(X, "iso", y, phi, th, xi, 0.1, inv_mass=np.array([4.0, 1.0, 0.0]))
    np.testing.assert_allclose(r["theta_prop"] - th, [0.06, -0.02, 0.0], atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_gaussian_integral_identity(n):
    g = np.random.default_rng(n)
    B = g.normal(size=(n, n))
    A = B @ B.T + 0.5 * np.eye(n)
    val = posterior.gaussian_integral(A, n_nodes={1: 401, 2: 201, 3: 121}[n])
    assert abs(val - np.linalg.det(A) ** -0.5) < 1e-10 * np.linalg.det(A) ** -0.5


def test_phi_marginal_is_posterior():
    # Integrating the extended density over phi gives P(theta) up to a theta-independent
    # constant (N/2) log(2 pi), checked across a theta grid at N = 2.
    X = np.array([[0.1], [0.55]])
    y = np.array([0.3, -0.8])
    diffs = []
    for la in (-1.0, 0.0, 0.7):
        for ll in (-1.5, -0.5, 0.4):
            th = np.array([la, ll, np.log(0.2)])
            diffs.append(posterior.log_phi_marginal(X, th, "iso", y, n_nodes=201) - posterior.log_posterior(X, th, "iso", y))
    np.testing.assert_allclose(diffs, math.log(2 * math.pi), atol=1e-10)


def test_log_posterior_two_points_closed_form():
    X = np.array([[0.0], [1.0]])
    y = np.array([1.0, 0.5])
    a, l, s2 = 1.5, 0.8, 0.1
    off = a * math.exp(-1.0 / (2 * l * l))
    A = np.array([[a + s2, off], [off, a + s2]])
    det = (a + s2) ** 2 - off ** 2
    quad = ((a + s2) * (y[0] ** 2 + y[1] ** 2) - 2 * off * y[0] * y[1]) / det
    expect = -0.5 * math.log(det) - 0.5 * quad
    assert abs(posterior.log_posterior(X, np.log([a, l, s2]), "iso", y) - expect) < 1e-13


# ---- implicit midpoint (Section 3.2.3) ------------------------------------------------------


def test_implicit_midpoint_is_the_cayley_map_on_a_quadratic_hamiltonian():
    # H = 1/2 theta^T Q theta + 1/2 pi^T pi: the implicit midpoint map is the Cayley transform
    # (I - dt/2 J H)^{-1} (I + dt/2 J H) of the linear flow, and it conserves H exactly
    g = np.random.default_rng(5)
    n = 4
    B = g.standard_normal((n, n))
    Q = B @ B.T + n * np.eye(n)
    th0, pi0 = g.standard_normal(n), g.standard_normal(n)
    dt = 0.3
    th1, pi1 = hmc.implicit_midpoint_step(lambda m: Q @ m, th0, pi0, dt)
    L = np.block([[np.zeros((n, n)), np.eye(n)], [-Q, np.zeros((n, n))]])   # d/dt (theta, pi)
    I2 = np.eye(2 * n)
    ref = np.linalg.solve(I2 - 0.5 * dt * L, (I2 + 0.5 * dt * L) @ np.concatenate([th0, pi0]))
    np.testing.assert_allclose(np.concatenate([th1, pi1]), ref, rtol=1e-12, atol=1e-12)
    H = lambda t, p: 0.5 * t @ Q @ t + 0.5 * p @ p
    assert abs(H(th1, pi1) - H(th0, pi0)) < 1e-12 * H(th0, pi0)


def _small_gp():
    X = I.uniform_points(40, 2, 21)
    y = I.y_sincos(X, 21)
    th = I.theta_iso(1.0, 0.3, 0.05)
    A = gp.a_matrix(X, th, "iso")
    phi = np.linalg.solve(np.linalg.cholesky(A).T, I.rng(21, I.P_XI).standard_normal(40))
    return X, y, th, phi


def test_implicit_midpoint_gp_reversible_and_second_order():
    X, y, th, phi = _small_gp()
    pi0 = np.array([0.3, -0.5, 0.2])
    th1, pi1 = hmc.implicit_midpoint(X, "iso", y, phi, th, pi0, 0.05, 3)
    thb, pib = hmc.implicit_midpoint(X, "iso", y, phi, th1, -pi1, 0.05, 3)
    np.testing.assert_allclose(thb, th, atol=1e-11)
    np.testing.assert_allclose(-pib, pi0, atol=1e-10)
    # the energy error of a symmetric second-order method falls by ~4 when dt halves
    errs = []
    for dt in (0.04, 0.02, 0.01):
        t, p = hmc.implicit_midpoint(X, "iso", y, phi, th, pi0, dt, int(round(0.08 / dt)))
        errs.append(abs(hmc.hamiltonian(X, t, "iso", y, phi, p) - hmc.hamiltonian(X, th, "iso", y, phi, pi0)))
    assert 2.5 < errs[0] / errs[1] < 6.0 and 2.5 < errs[1] / errs[2] < 6.0, errs


def test_implicit_midpoint_satisfies_its_defining_equations():
    X, y, th, phi = _small_gp()
    pi0 = np.array([0.1, 0.4, -0.3])
    dt = 0.07
    th1, pi1 = hmc.implicit_midpoint(X, "iso", y, phi, th, pi0, dt, 1)
    m = 0.5 * (th + th1)
    np.testing.assert_allclose(th1, th + dt * 0.5 * (pi0 + pi1), atol=1e-13)
    # pi_1 = pi_0 - dt F(m), F by central differences of u(theta, x) at x = A(m)^{-1} y frozen
    x = hmc.solve(X, m, "iso", y)
    h = 1e-6
    F = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        up = -0.5 * x @ gp.a_matrix(X, m + e, "iso") @ x + 0.5 * phi @ gp.a_matrix(X, m + e, "iso") @ phi
        um = -0.5 * x @ gp.a_matrix(X, m - e, "iso") @ x + 0.5 * phi @ gp.a_matrix(X, m - e, "iso") @ phi
        F[k] = (up - um) / (2 * h)
    np.testing.assert_allclose(pi1, pi0 - dt * F, atol=1e-7)


# ---- random-walk Metropolis (the RWM update of theta) ---------------------------------------


def _one_point_potential(th, y, phi):
    # N = 1: A = alpha + sigma^2 whatever the length-scale, so
    # U = 1/2 y^2 / (alpha + sigma^2) + 1/2 phi^2 (alpha + sigma^2)
    a = math.exp(th[0]) + math.exp(th[2])
    return 0.5 * y * y / a + 0.5 * phi * phi * a


def test_rwm_energies_and_proposal_one_point_closed_form():
    X = np.array([[0.3]])
    y, phi = 0.7, -1.3
    th0 = np.array([0.2, -0.4, math.log(0.3)])
    xi = np.array([0.5, 2.0, -1.5])
    r = hmc.rwm_update(X, "iso", np.array([y]), np.array([phi]), th0, xi, 0.3)
    prop = th0 + 0.3 * xi
    assert abs(r["U0"] - _one_point_potential(th0, y, phi)) < 1e-13
    assert abs(r["U1"] - _one_point_potential(prop, y, phi)) < 1e-13
    np.testing.assert_allclose(r["theta"], prop, rtol=0, atol=1e-15)
    assert r["accepted"]


def test_rwm_acceptance_frequency_is_min_one_exp_energy_drop():
    # over a fine grid of uniforms the accepted fraction is min(1, exp(U0 - U1)): exp of the
    # energy drop when the proposal goes uphill, 1 when it goes downhill
    X = np.array([[0.3]])
    y, phi = 1.1, 0.4
    th0 = np.array([0.0, 0.0, math.log(0.5)])
    K = 20000
    us = (np.arange(K) + 0.5) / K
    for xi in (np.array([1.0, 0.0, 0.0]), np.array([-1.0, 0.0, -1.0]), np.array([0.3, 0.0, 0.8])):
        u0 = _one_point_potential(th0, y, phi)
        u1 = _one_point_potential(th0 + 0.5 * xi, y, phi)
        frac = np.mean([hmc.rwm_update(X, "iso", np.array([y]), np.array([phi]), th0, xi, 0.5, u=u)["accepted"]
                        for u in us[::20]])
        assert abs(frac - min(1.0, math.exp(u0 - u1))) < 2e-3, (xi, frac, u0, u1)


def test_rwm_reject_restores_and_zero_step_always_accepts():
    X, y, th, phi = _problem()
    xi = np.array([2.0, -1.0, 0.5])
    r = hmc.rwm_update(X, "iso", y, phi, th, xi, 0.0, u=1.0 - 1e-15)
    assert r["accepted"] and r["U0"] == r["U1"]
    r = hmc.rwm_update(X, "iso", y, phi, th, xi, 0.4, u=1.0 - 1e-15)
    if r["U1"] > r["U0"]:
        assert not r["accepted"]
        np.testing.assert_array_equal(r["theta"], th)
