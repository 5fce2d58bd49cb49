"""Pins of the oracle's randomized Nystrom preconditioner and preconditioned CG.

Independent checks: a kernel of exact low rank is recovered exactly; a full-rank sketch
recovers K itself (so P^{-1}(A + lambda) is a multiple of I and PCG converges in one step);
K - K_hat is positive semidefinite (the Nystrom approximation never overshoots); PCG solutions
equal a dense solve; and a good preconditioner cuts the iteration count.
"""
import numpy as np

from oracle import gp, precond


def _setup(n=120, d=2, seed=0, ell=0.3, sigma2=1e-3):
    g = np.random.default_rng([seed, 900])
    X = g.uniform(0.0, 1.0, size=(n, d))
    th = np.array([0.0, np.log(ell), np.log(sigma2)])
    return X, th, g


def test_exact_on_rank_one_kernel():
    # l -> infinity: K = alpha 1 1^T has rank 1; any sketch of rank >= 1 recovers it
    X, _, g = _setup()
    th = np.array([np.log(2.0), np.log(1e6), np.log(1e-2)])
    U, lam = precond.nystrom(X, th, "iso", g.standard_normal((120, 3)))
    K = gp.a_matrix(X, th, "iso", no_noise=True)
    np.testing.assert_allclose(U @ np.diag(lam) @ U.T, K, atol=1e-8 * np.abs(K).max())
    assert abs(lam[0] - 2.0 * 120) < 1e-6 * 240 and np.all(lam[1:] < 1e-6)


def test_full_rank_sketch_recovers_k_and_one_step_pcg():
    n = 60
    X, th, g = _setup(n=n, ell=0.2, sigma2=1e-2)
    U, lam = precond.nystrom(X, th, "iso", g.standard_normal((n, n)))
    K = gp.a_matrix(X, th, "iso", no_noise=True)
    np.testing.assert_allclose(U @ np.diag(lam) @ U.T, K, atol=1e-9 * np.abs(K).max())
    b = g.standard_normal(n)
    x, it = precond.pcg(X, th, "iso", b, shift=0.3, U=U, lam=lam, tol=1e-10)
    assert it <= 2
    np.testing.assert_allclose(x, np.linalg.solve(gp.a_matrix(X, th, "iso") + 0.3 * np.eye(n), b), rtol=1e-8)


def test_nystrom_never_overshoots():
    X, th, g = _setup(n=150, ell=0.15)
    U, lam = precond.nystrom(X, th, "iso", g.standard_normal((150, 12)))
    K = gp.a_matrix(X, th, "iso", no_noise=True)
    ev = np.linalg.eigvalsh(K - U @ np.diag(lam) @ U.T)
    assert ev[0] > -1e-9 * np.abs(K).max()
    # K_hat <= K in the Loewner order, so its eigenvalues interlace from below
    top = np.linalg.eigvalsh(K)[::-1][:12]
    assert np.all(lam <= top * (1 + 1e-9))


def test_error_within_the_randomized_low_rank_bound():
    # a smooth kernel (l = 0.6 on [0,1]^2) has fast spectral decay.  For a Gaussian sketch of
    # l = k + p columns the expected spectral error is at most
    #   (1 + 2k/(p-1)) lam_{k+1} + (2 e sqrt(l) / p) (sum_{j>k} lam_j^2)^{1/2}
    # (Halko-Martinsson-Tropp); with k = p = 6 it must hold here, and the top eigenvalues follow
    X, th, g = _setup(n=150, ell=0.6)
    K = gp.a_matrix(X, th, "iso", no_noise=True)
    U, lam = precond.nystrom(X, th, "iso", g.standard_normal((150, 12)))
    ev = np.linalg.eigvalsh(K)[::-1]
    k, p = 6, 6
    bound = (1 + 2 * k / (p - 1)) * ev[k] + 2 * np.e * np.sqrt(k + p) / p * np.sqrt(np.sum(ev[k:] ** 2))
    err = np.linalg.eigvalsh(K - U @ np.diag(lam) @ U.T)[-1]
    assert err <= bound, (err, bound)
    assert np.all(np.abs(lam[:3] - ev[:3]) <= err + 1e-12)


def test_pcg_matches_dense_solve_and_reduces_iterations():
    n = 200
    X, th, g = _setup(n=n, ell=0.3, sigma2=1e-4)
    b = g.standard_normal(n)
    A = gp.a_matrix(X, th, "iso")
    x0, it0 = precond.pcg(X, th, "iso", b, tol=1e-10)
    U, lam = precond.nystrom(X, th, "iso", g.standard_normal((n, 30)))
    x1, it1 = precond.pcg(X, th, "iso", b, U=U, lam=lam, tol=1e-10)
    ref = np.linalg.solve(A, b)
    np.testing.assert_allclose(x0, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())
    np.testing.assert_allclose(x1, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())
    assert it1 < it0 / 3, (it0, it1)


def test_preconditioner_is_spd_and_identity_off_the_sketch():
    n = 80
    X, th, g = _setup(n=n)
    U, lam = precond.nystrom(X, th, "iso", g.standard_normal((n, 6)))
    P = precond.precond_apply(U, lam, 0.01, np.eye(n))
    np.testing.assert_allclose(P, P.T, atol=1e-12)
    assert np.linalg.eigvalsh(P)[0] > 0
    # a vector orthogonal to range(U) passes unchanged
    v = g.standard_normal(n)
    v -= U @ (U.T @ v)
    np.testing.assert_allclose(precond.precond_apply(U, lam, 0.01, v), v, atol=1e-12)
