"""Randomized Nystrom preconditioner and preconditioned CG (Section 3.1 after eq. pex; Section
3.2.3; Section 4.1) against the oracle.

The factor U diag(lam) U^T depends only on range(Omega), so it is compared as a matrix (the
columns of U are unique only up to sign).  FP64 tolerances follow the oracle's own arithmetic
(1e-9 on the factor, 1e-9 on solves at tol 1e-12); FP32 factors are compared at
20 eps32 lam_1 / lam_l, the sketch's float rounding amplified by the Cholesky step.
"""
import numpy as np
import pytest
import torch

from oracle import gp as ogp, precond as opre
from paper_2412_20884_amd import gpk
from tests.gpu_util import host, rounded, to_dev

pytestmark = pytest.mark.gpu


def _problem(n, d, seed, kind="iso", ell=0.3, sigma2=1e-3, r=2):
    g = np.random.default_rng([seed, 611])
    X = g.uniform(0.0, 1.0, size=(n, d))
    if kind == "iso":
        th = np.array([0.1, np.log(ell), np.log(sigma2)])
    else:
        th = np.concatenate([[0.1], np.log(ell * np.exp(0.3 * g.standard_normal(d))), [np.log(sigma2)]])
    return X, th, g.standard_normal((n, r)), g


@pytest.mark.parametrize("kind,d,rank", [("iso", 2, 5), ("ard", 4, 40), ("iso", 3, 130)])
def test_nystrom_factor_f64(kind, d, rank):
    n = 900
    X, th, _, g = _problem(n, d, rank, kind)
    om = g.standard_normal((n, rank))
    U, lam = gpk.nystrom(to_dev(X, torch.float64), to_dev(th, torch.float64), to_dev(om, torch.float64), kind)
    torch.cuda.synchronize()
    Uo, lo = opre.nystrom(X, th, kind, om)
    U, lam = host(U), host(lam)
    Kg = U @ np.diag(lam) @ U.T
    Ko = Uo @ np.diag(lo) @ Uo.T
    assert np.linalg.norm(Kg - Ko) < 1e-9 * np.linalg.norm(Ko)
    assert np.max(np.abs(lam - lo)) < 1e-9 * lo[0]
    assert np.all(np.diff(lam) <= 0)
    np.testing.assert_allclose(U.T @ U, np.eye(rank), atol=1e-10)


def test_nystrom_factor_f32_and_cheb():
    n, rank = 1500, 20
    X, th, _, g = _problem(n, 2, 3)
    om = g.standard_normal((n, rank))
    Xr, omr = rounded(X, torch.float32), rounded(om, torch.float32)
    U, lam = gpk.nystrom(to_dev(Xr, torch.float32), to_dev(th, torch.float64), to_dev(omr, torch.float32), "iso")
    torch.cuda.synchronize()
    Uo, lo = opre.nystrom(Xr, th, "iso", omr)
    U, lam = host(U), host(lam)
    Ko = Uo @ np.diag(lo) @ Uo.T
    # float32 sketch (Y = K Q to ~eps32), amplified by the condition lam_1 / lam_l of Q^T K Q
    # through the Cholesky factor and C^{-1}
    bound = 20 * 2.0 ** -24 * lo[0] / lo[-1]
    assert np.linalg.norm(U @ np.diag(lam) @ U.T - Ko) < bound * np.linalg.norm(Ko)
    # the Chebyshev-amplitude kernel goes through the same construction
    Xc = 2.0 * X - 1.0
    thc = np.array([0.2, -0.1, 0.05, 0.1, np.log(0.4), np.log(1e-2)])
    U2, l2 = gpk.nystrom(to_dev(Xc, torch.float64), to_dev(thc, torch.float64), to_dev(om, torch.float64),
                         "cheb", n_cheb=2)
    torch.cuda.synchronize()
    Uo2, lo2 = opre.nystrom(Xc, thc, "cheb", om)
    Ko2 = Uo2 @ np.diag(lo2) @ Uo2.T
    assert np.linalg.norm(host(U2) @ np.diag(host(l2)) @ host(U2).T - Ko2) < 1e-9 * np.linalg.norm(Ko2)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("rank", [0, 25])
def test_pcg_solve_with_shifts(dtype, rank):
    n = 1200
    X, th, B, g = _problem(n, 2, 7, sigma2=1e-3, r=3)
    shift = np.array([0.0, 0.05, 1.3])
    X, B = rounded(X, dtype), rounded(B, dtype)
    Xd, thd = to_dev(X, dtype), to_dev(th, torch.float64)
    U = lam = None
    if rank:
        U, lam = gpk.nystrom(Xd, thd, to_dev(rounded(g.standard_normal((n, rank)), dtype), dtype), "iso")
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    res = gpk.pcg_solve(Xd, thd, to_dev(B, dtype), "iso", col_shift=to_dev(shift, torch.float64), U=U,
                        lam=lam, tol=tol, maxit=20000)
    torch.cuda.synchronize()
    assert np.all(host(res["status"]) == 0), host(res["status"])
    A = ogp.a_matrix(X, th, "iso")
    x = host(res["x"])
    for c in range(3):
        ref = np.linalg.solve(A + shift[c] * np.eye(n), B[:, c])
        cond = np.linalg.cond(A + shift[c] * np.eye(n))
        bound = 1e-9 if dtype == torch.float64 else min(1e-1, 20 * cond * 2.0 ** -24)
        assert np.linalg.norm(x[:, c] - ref) < bound * np.linalg.norm(ref), (c, cond)


def test_preconditioner_cuts_iterations_and_matches_oracle_pcg():
    n = 1500
    X, th, B, g = _problem(n, 2, 11, ell=0.25, sigma2=1e-4, r=1)
    om = g.standard_normal((n, 60))
    Xd, thd = to_dev(X, torch.float64), to_dev(th, torch.float64)
    U, lam = gpk.nystrom(Xd, thd, to_dev(om, torch.float64), "iso")
    plain = gpk.pcg_solve(Xd, thd, to_dev(B[:, 0], torch.float64), "iso", tol=1e-10, maxit=20000)
    pre = gpk.pcg_solve(Xd, thd, to_dev(B[:, 0], torch.float64), "iso", U=U, lam=lam, tol=1e-10, maxit=20000)
    torch.cuda.synchronize()
    it_plain, it_pre = int(plain["iters"][0]), int(pre["iters"][0])
    Uo, lo = opre.nystrom(X, th, "iso", om)
    xo, it_o = opre.pcg(X, th, "iso", B[:, 0], U=Uo, lam=lo, tol=1e-10)
    _, it_o0 = opre.pcg(X, th, "iso", B[:, 0], tol=1e-10)
    print(f"CG {it_plain} (oracle {it_o0}) vs Nystrom-PCG {it_pre} (oracle {it_o})")
    assert it_pre < it_plain / 3
    assert abs(it_pre - it_o) <= max(2, 0.05 * it_o) and abs(it_plain - it_o0) <= max(3, 0.05 * it_o0)
    np.testing.assert_allclose(host(pre["x"]), xo, rtol=0, atol=1e-7 * np.abs(xo).max())


def test_pcg_warm_start_and_maxit():
    n = 600
    X, th, B, _ = _problem(n, 2, 13, r=2)
    A = ogp.a_matrix(X, th, "iso")
    exact = np.linalg.solve(A, B)
    Xd, thd, Bd = to_dev(X, torch.float64), to_dev(th, torch.float64), to_dev(B, torch.float64)
    warm = gpk.pcg_solve(Xd, thd, Bd, "iso", x0=to_dev(exact, torch.float64), tol=1e-8)
    short = gpk.pcg_solve(Xd, thd, Bd, "iso", tol=1e-14, maxit=3)
    torch.cuda.synchronize()
    assert np.all(host(warm["iters"]) == 0) and np.all(host(warm["status"]) == 0)
    assert np.all(host(short["status"]) == gpk.CG_MAXIT) and np.all(host(short["iters"]) == 3)
    # a replayed group of four iterations and three single ones: still exactly the limit
    seven = gpk.pcg_solve(Xd, thd, Bd, "iso", tol=1e-14, maxit=7)
    torch.cuda.synchronize()
    assert np.all(host(seven["status"]) == gpk.CG_MAXIT) and np.all(host(seven["iters"]) == 7)
