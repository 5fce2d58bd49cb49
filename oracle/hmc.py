"""Oracle: exact solve, potential, force, leapfrog, Hamiltonian and accept test (FP64, CPU).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Definitions followed (paper section / equation):
  * U_phi(theta) = S(theta) + 1/2 y^T A(theta)^{-1} y + 1/2 phi^T A(theta) phi   (Section 3.2, eq. U)
  * x_theta solves A(theta) x = y                                              (eq. xtheta)
  * u_phi(theta, x) = S(theta) - 1/2 x^T A(theta) x + 1/2 phi^T A(theta) phi   (eq. u)
    and the force F_phi(theta) = grad_theta u_phi(theta, x) at x = x_theta with x held fixed
    (Section 3.2.1, the frozen-x evaluation).
  * H_phi(theta, pi) = U_phi(theta) + 1/2 pi^T M^{-1} pi (Section 3.2).  The paper's runs use
    M = I; a diagonal M^{-1} = diag(inv_mass) is accepted here, and a zero entry of inv_mass is
    the limit of an infinite mass: that component of theta never moves and its momentum adds no
    kinetic energy (used to hold a hyperparameter fixed).
  * Stormer-Verlet step (Section 3.2.2), drift-kick-drift with the force at the half step:
        theta_1/2 = theta_0 + dt/2 * M^{-1} pi_0
        pi_1      = pi_0 - dt * F(theta_1/2)
        theta_1   = theta_1/2 + dt/2 * M^{-1} pi_1
    (the printed kick has pi_1 on both sides; the reading used here starts from pi_0).
  * Metropolis test (Section 3.2, step (3); Algorithm 1): accept with probability
    min(1, exp(H_0 - H_1)); with a supplied uniform u the decision is  log u <= H_0 - H_1.
  * Random-walk Metropolis (the RWM alternative for the update of theta in Section 3; proposal
    and rule as stated at the start of Section 4): theta' = theta + dt * xi, xi ~ N(0, I),
    accepted with probability min(1, exp(U_phi(theta) - U_phi(theta'))).  With a diagonal
    inverse mass the step is dt * sqrt(inv_mass) * xi (proposal covariance dt^2 M^{-1}).

The linear solve here is an exact Cholesky solve: the oracle never iterates.  The prior is
flat (S = 0) unless a callable is supplied.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from . import gp


def solve(X, theta, kind, y):
    """x_theta = A(theta)^{-1} y by Cholesky (eq. xtheta)."""
    A = gp.a_matrix(X, theta, kind)
    return cho_solve(cho_factor(A, lower=True), np.asarray(y, dtype=np.float64))


def potential(X, theta, kind, y, phi, prior=None):
    """U_phi(theta) (eq. U); `prior` returns S(theta) = -log p(theta) (flat if None)."""
    y = np.asarray(y, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    A = gp.a_matrix(X, theta, kind)
    x = cho_solve(cho_factor(A, lower=True), y)
    s = 0.0 if prior is None else float(prior(theta))
    return s + 0.5 * float(y @ x) + 0.5 * float(phi @ (A @ phi))


def potential_at(X, theta, kind, y, phi, x):
    """U_phi(theta) with y^T A^{-1} y replaced by its variational form 2 y^T x - x^T A x.

    For the exact solution x = A^{-1} y both forms agree; for an approximate x the error of
    the variational form is r^T A^{-1} r with r = y - A x (second order in the residual).
    """
    A = gp.a_matrix(X, theta, kind)
    x = np.asarray(x, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    return 0.5 * (2.0 * float(y @ x) - float(x @ (A @ x))) + 0.5 * float(phi @ (A @ phi))


def force(X, theta, kind, y, phi, grad_prior=None, x=None):
    """F_phi(theta) = grad_theta u_phi(theta, x)|_{x = x_theta}, Section 3.2.1.

    u_phi = S - 1/2 x^T A x + 1/2 phi^T A phi, so with U = V = [x | phi] and weights
    (-1/2, +1/2) this is one quadratic-form gradient.
    """
    if x is None:
        x = solve(X, theta, kind, y)
    Z = np.stack([np.asarray(x, np.float64), np.asarray(phi, np.float64)], axis=1)
    g = gp.quadform_grad(X, theta, kind, Z, Z, w=np.array([-0.5, 0.5]))["grad"]
    if grad_prior is not None:
        g = g + np.asarray(grad_prior(theta), dtype=np.float64)
    return g


def _minv(inv_mass, n):
    return np.ones(n) if inv_mass is None else np.asarray(inv_mass, dtype=np.float64)


def hamiltonian(X, theta, kind, y, phi, pi, prior=None, inv_mass=None):
    """H_phi(theta, pi) = U_phi(theta) + 1/2 pi^T M^{-1} pi, Section 3.2 (M = I by default)."""
    pi = np.asarray(pi, dtype=np.float64)
    return potential(X, theta, kind, y, phi, prior) + 0.5 * float(pi @ (_minv(inv_mass, len(pi)) * pi))


def leapfrog(X, kind, y, phi, theta0, pi0, dt, n_steps, grad_prior=None, history=False,
             inv_mass=None):
    """[S_{phi,dt}]^{n_steps}(theta0, pi0): drift-kick-drift Stormer-Verlet, Section 3.2.2."""
    theta = np.array(theta0, dtype=np.float64)
    pi = np.array(pi0, dtype=np.float64)
    minv = _minv(inv_mass, len(pi))
    hist = []
    for _ in range(n_steps):
        theta_half = theta + 0.5 * dt * (minv * pi)
        pi = pi - dt * force(X, theta_half, kind, y, phi, grad_prior)
        theta = theta_half + 0.5 * dt * (minv * pi)
        if history:
            hist.append((theta.copy(), pi.copy()))
    if history:
        return theta, pi, hist
    return theta, pi


def accept(H0, H1, u):
    """Metropolis decision of Algorithm 1: accept iff u <= exp(H0 - H1), as log u <= H0 - H1."""
    if u <= 0.0:
        return True
    return bool(np.log(u) <= H0 - H1)


def trajectory(X, kind, y, phi, theta0, pi0, dt, n_steps, u=None, prior=None, grad_prior=None,
               inv_mass=None):
    """One HMC update of theta given phi (Algorithm 1, steps 5-10, with pi supplied).

    Returns dict(theta, pi, theta_prop, pi_prop, H0, H1, accepted).  With u None no
    decision is taken and the proposal is returned as accepted.
    """
    H0 = hamiltonian(X, theta0, kind, y, phi, pi0, prior, inv_mass)
    th, p = leapfrog(X, kind, y, phi, theta0, pi0, dt, n_steps, grad_prior, inv_mass=inv_mass)
    H1 = hamiltonian(X, th, kind, y, phi, p, prior, inv_mass)
    ok = True if u is None else accept(H0, H1, u)
    return {
        "theta": th if ok else np.array(theta0, dtype=np.float64),
        "pi": p if ok else np.array(pi0, dtype=np.float64),
        "theta_prop": th,
        "pi_prop": p,
        "H0": H0,
        "H1": H1,
        "accepted": ok,
    }


def rwm_update(X, kind, y, phi, theta0, xi, dt, u=None, prior=None, inv_mass=None):
    """One random-walk Metropolis update of theta given phi (the RWM alternative of Section 3,
    with the proposal and acceptance rule stated at the start of Section 4): the proposal is
    theta' = theta0 + dt * xi with xi ~ N(0, I) supplied, accepted with probability
    min(1, exp(U_phi(theta0) - U_phi(theta'))); with a supplied uniform u the decision is
    log u <= U_0 - U_1, and with u None the proposal is returned as accepted.

    Returns dict(theta, theta_prop, U0, U1, accepted).
    """
    theta0 = np.asarray(theta0, dtype=np.float64)
    prop = theta0 + dt * np.sqrt(_minv(inv_mass, len(theta0))) * np.asarray(xi, dtype=np.float64)
    U0 = potential(X, theta0, kind, y, phi, prior)
    U1 = potential(X, prop, kind, y, phi, prior)
    ok = True if u is None else accept(U0, U1, u)
    return {"theta": prop if ok else theta0.copy(), "theta_prop": prop, "U0": U0, "U1": U1,
            "accepted": ok}


# ---- implicit midpoint integrator (Section 3.2.3) ------------------------------------------


def implicit_midpoint_step(force_fn, theta0, pi0, dt, tol=1e-14, maxit=10000):
    """One step of the 1-stage Gauss-Legendre (implicit midpoint) integrator, eq. (implicitsystem):
        theta_1 = theta_0 + dt (pi_0 + pi_1) / 2,   pi_1 = pi_0 - dt F((theta_0 + theta_1) / 2).
    Eliminating theta_1 and pi_1 leaves the midpoint m = (theta_0 + theta_1)/2 as the fixed point of
        m = theta_0 + dt/2 pi_0 - dt^2/4 F(m),
    iterated here until the update is below tol (relative); raises if it does not converge.
    """
    theta0 = np.asarray(theta0, dtype=np.float64)
    pi0 = np.asarray(pi0, dtype=np.float64)
    m = theta0 + 0.5 * dt * pi0
    for _ in range(maxit):
        m_new = theta0 + 0.5 * dt * pi0 - 0.25 * dt * dt * np.asarray(force_fn(m), dtype=np.float64)
        done = np.max(np.abs(m_new - m)) <= tol * (1.0 + np.max(np.abs(m_new)))
        m = m_new
        if done:
            pi1 = pi0 - dt * np.asarray(force_fn(m), dtype=np.float64)
            return 2.0 * m - theta0, pi1
    raise RuntimeError("implicit midpoint fixed point did not converge")


def implicit_midpoint(X, kind, y, phi, theta0, pi0, dt, n_steps, grad_prior=None, tol=1e-14):
    """[implicit midpoint]^{n_steps}(theta0, pi0) with the exact-solve force: at the solution the
    third equation of (implicitsystem), A(m) x = y, holds exactly because F is evaluated at
    x = A(m)^{-1} y (Cholesky)."""
    theta = np.array(theta0, dtype=np.float64)
    pi = np.array(pi0, dtype=np.float64)
    for _ in range(n_steps):
        theta, pi = implicit_midpoint_step(lambda m: force(X, m, kind, y, phi, grad_prior), theta, pi,
                                           dt, tol=tol)
    return theta, pi
