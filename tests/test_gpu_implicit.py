"""Implicit midpoint HMC (Section 3.2.3) with Anderson acceleration (Appendix B) against the
oracle's implicit midpoint, whose midpoint equation is solved to machine precision with exact
(Cholesky) solves.  The GPU stops its fixed-point iteration at tol on (theta, pi) and at cg_tol
on the linear part, so in FP64 with tol 1e-12 and cg_tol 1e-12 the trajectories agree to 1e-8.
"""
import numpy as np
import pytest
import torch

from oracle import gp as ogp, hmc as ohmc, precond as opre
from paper_2412_20884_amd import gpk, inputs as I
from tests.gpu_util import host, to_dev

pytestmark = pytest.mark.gpu


def _chain(n, seed, kind="iso", d=2, sigma2=0.05):
    X = I.uniform_points(n, d, seed)
    y = I.y_sincos(X, seed) if d == 2 else I.y_prodcos(X, seed)
    th = I.theta_iso(1.0, 0.3, sigma2) if kind == "iso" else I.theta_ard_loguniform(d, 0.3, 1.0, seed, sigma2=sigma2)
    A = ogp.a_matrix(X, th, kind)
    phi = np.linalg.solve(np.linalg.cholesky(A).T, I.rng(seed, I.P_XI).standard_normal(n))
    pi0 = I.rng(seed, I.P_PI).standard_normal(len(th))
    return X, y, th, phi, pi0


def _run(X, y, th, phi, pi0, kind, dtype, **kw):
    thd, pid = to_dev(th, torch.float64), to_dev(pi0, torch.float64)
    xw = torch.zeros(len(y), dtype=dtype, device="cuda:0")
    r = gpk.hmc_implicit(to_dev(X, dtype), to_dev(y, dtype), to_dev(phi, dtype), thd, pid, xw, kind, **kw)
    torch.cuda.synchronize()
    return host(thd), host(pid), {k: host(v)[0] if v.dtype == torch.float64 else int(v[0]) for k, v in r.items()}, xw


@pytest.mark.parametrize("kind,sigma2,rank", [("iso", 0.3, 0), ("ard", 0.3, 0), ("iso", 0.05, 30),
                                              ("ard", 0.05, 30)])
def test_implicit_matches_oracle_fp64(kind, sigma2, rank):
    X, y, th, phi, pi0 = _chain(300, 31, kind, d=2 if kind == "iso" else 3, sigma2=sigma2)
    U = lam = None
    if rank:  # the Nystrom-based R of Section 3.2.3 for the worse-conditioned problems
        U, lam = gpk.nystrom(to_dev(X, torch.float64), to_dev(th, torch.float64),
                             to_dev(I.normal_matrix(300, rank, 31, I.P_V), torch.float64), kind)
    th1, pi1, r, xw = _run(X, y, th, phi, pi0, kind, torch.float64, n_steps=3, dt=0.05, history=10,
                           tol=1e-12, maxit=3000, cg_tol=1e-12, cg_maxit=5000, U=U, lam=lam)
    tho, pio = ohmc.implicit_midpoint(X, kind, y, phi, th, pi0, 0.05, 3)
    print(f"implicit {kind} sigma2={sigma2} rank={rank}: {r['iters']} fixed-point iterations")
    assert r["status"] == 0, r
    assert np.max(np.abs(th1 - tho)) < 1e-8 and np.max(np.abs(pi1 - pio)) < 1e-8
    H0 = ohmc.hamiltonian(X, th, kind, y, phi, pi0)
    H1 = ohmc.hamiltonian(X, tho, kind, y, phi, pio)
    assert abs(r["H0"] - H0) < 1e-9 * abs(H0) and abs(r["H1"] - H1) < 1e-9 * abs(H1)
    np.testing.assert_allclose(host(xw), ohmc.solve(X, tho, kind, y), atol=1e-8)


def test_anderson_beats_picard_and_both_agree():
    # plain fixed-point iteration contracts the linear part only by 1 - lambda_min / c per step,
    # so the comparison runs on a well-conditioned problem (sigma^2 = 1)
    X, y, th, phi, pi0 = _chain(400, 5, sigma2=1.0)
    kw = dict(n_steps=2, dt=0.08, tol=1e-9, maxit=8000, cg_tol=1e-9, cg_maxit=5000)
    thp, pip, rp, _ = _run(X, y, th, phi, pi0, "iso", torch.float64, history=0, **kw)
    tha, pia, ra, _ = _run(X, y, th, phi, pi0, "iso", torch.float64, history=10, **kw)
    print(f"fixed-point iterations: Picard {rp['iters']}, Anderson(10) {ra['iters']}")
    assert rp["status"] == 0 and ra["status"] == 0
    assert ra["iters"] < rp["iters"] / 2
    assert np.max(np.abs(thp - tha)) < 1e-7 and np.max(np.abs(pip - pia)) < 1e-7


def test_implicit_float32_nystrom_endpoints_and_flags():
    X, y, th, phi, pi0 = _chain(1500, 9)
    Xd = to_dev(X, torch.float32)
    om = to_dev(I.normal_matrix(1500, 20, 9, I.P_V), torch.float32)
    U, lam = gpk.nystrom(Xd, to_dev(th, torch.float64), om, "iso")
    thd, pid = to_dev(th, torch.float64), to_dev(pi0, torch.float64)
    xw = torch.zeros(1500, dtype=torch.float32, device="cuda:0")
    r = gpk.hmc_implicit(Xd, to_dev(y, torch.float32), to_dev(phi, torch.float32), thd, pid, xw, "iso",
                         n_steps=3, dt=0.05, history=10, tol=1e-4, maxit=2000, cg_tol=1e-4, U=U, lam=lam)
    torch.cuda.synchronize()
    tho, pio = ohmc.implicit_midpoint(X, "iso", y, phi, th, pi0, 0.05, 3)
    # In float32 the fixed point recomputes y - A(m) x and the force from float products each
    # iteration: their rounding (relative to |A||x| and to the N-scale quadratic forms, not to |y|
    # or F) sets floors near 1e-5, hence tolerances of 1e-4 here
    assert int(r["status"][0]) == 0, int(r["iters"][0])
    assert np.max(np.abs(host(thd) - tho)) < 2e-3
    # maxit too small: flagged and rejected, start state restored
    thd2, pid2 = to_dev(th, torch.float64), to_dev(pi0, torch.float64)
    r2 = gpk.hmc_implicit(Xd, to_dev(y, torch.float32), to_dev(phi, torch.float32), thd2, pid2,
                          torch.zeros(1500, dtype=torch.float32, device="cuda:0"), "iso", n_steps=2,
                          dt=0.05, history=10, tol=1e-12, maxit=2, cg_tol=1e-6,
                          u=to_dev(np.array([0.5]), torch.float64))
    torch.cuda.synchronize()
    assert int(r2["status"][0]) & gpk.CHAIN_FP_MAXIT and int(r2["accepted"][0]) == 0
    np.testing.assert_array_equal(host(thd2), th)
    np.testing.assert_array_equal(host(pid2), pi0)
    # the iterations run as replays of a captured group of four: a limit that is not a multiple
    # of four still stops at the limit (2, then 6 = one group and half of the next)
    assert int(r2["iters"][0]) == 2
    r3 = gpk.hmc_implicit(Xd, to_dev(y, torch.float32), to_dev(phi, torch.float32),
                          to_dev(th, torch.float64), to_dev(pi0, torch.float64),
                          torch.zeros(1500, dtype=torch.float32, device="cuda:0"), "iso", n_steps=2,
                          dt=0.05, history=10, tol=1e-12, maxit=6, cg_tol=1e-6)
    torch.cuda.synchronize()
    assert int(r3["status"][0]) & gpk.CHAIN_FP_MAXIT and int(r3["iters"][0]) == 6


def test_implicit_cheb_kernel():
    """The paper's E1 setting (Section 4.1: N = 10 equispaced on [-1, 1), d = 1, N_cheb = 2,
    2 l^2 = 1, sigma^2 = 0.1, y = 1) with its implicit step dt = 0.15, N_int = 3."""
    n = 10
    X = (-1.0 + 2.0 * np.arange(n) / n)[:, None]
    y = np.ones(n)
    th = np.array([0.01, 0.01, np.log(np.sqrt(0.5)), np.log(0.1)])
    A = ogp.a_matrix(X, th, "cheb")
    phi = np.linalg.solve(np.linalg.cholesky(A).T, I.rng(2, I.P_XI).standard_normal(n))
    pi0 = I.rng(2, I.P_PI).standard_normal(4)
    th1, pi1, r, _ = _run(X, y, th, phi, pi0, "cheb", torch.float64, n_steps=3, dt=0.15, history=10,
                          tol=1e-13, maxit=400, cg_tol=1e-13, n_cheb=2)
    tho, pio = ohmc.implicit_midpoint(X, "cheb", y, phi, th, pi0, 0.15, 3)
    assert r["status"] == 0
    assert np.max(np.abs(th1 - tho)) < 1e-8 and np.max(np.abs(pi1 - pio)) < 1e-8
