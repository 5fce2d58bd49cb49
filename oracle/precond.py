"""Oracle: randomized Nystrom preconditioner and preconditioned CG (FP64, CPU).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Definitions followed (paper section):
  * Section 3.1 (after eq. pex) and Section 3.2.3: a low-rank factorization of K(theta)
    (eq. kernmat), K ~ U diag(lam) U^T, gives an approximate inverse of A + lambda I =
    K + (sigma^2 + lambda) I through the Woodbury identity, one factorization for every shift;
    the paper uses the randomized Nystrom construction of Frangella, Tropp and Udell (rank 5 in
    Section 4.1, rank 500 in Section 4.3).  The steps, in that construction's order:
        Q = orth(Omega)                     Omega an n x l Gaussian test matrix
        Y = K Q
        nu = sqrt(n) eps |Y|_F              a stabilising shift
        Y_nu = Y + nu Q
        C^T C = Q^T Y_nu                    Cholesky
        B = Y_nu C^{-1}
        B = U S V^T                         thin SVD
        lam = max(0, S^2 - nu)
  * The preconditioner for A + lambda I, with mu = sigma^2 + lambda:
        P^{-1} = U diag((lam_l + mu) / (lam + mu)) U^T + (I - U U^T).
  * Conjugate gradients for each column with P^{-1} (textbook preconditioned CG).
"""
from __future__ import annotations

import numpy as np

from . import gp


def nystrom(X, theta, kind, omega):
    """(U, lam): the randomized Nystrom approximation K ~ U diag(lam) U^T for test matrix omega."""
    X = np.asarray(X, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    n = X.shape[0]
    Q, _ = np.linalg.qr(omega)
    Y = gp.matvec(X, theta, kind, Q, no_noise=True)
    nu = np.sqrt(n) * np.finfo(np.float64).eps * np.linalg.norm(Y)
    Ynu = Y + nu * Q
    C = np.linalg.cholesky(Q.T @ Ynu).T            # upper: C^T C = Q^T Y_nu
    B = np.linalg.solve(C.T, Ynu.T).T              # B = Y_nu C^{-1}
    U, S, _ = np.linalg.svd(B, full_matrices=False)
    lam = np.maximum(0.0, S * S - nu)
    return U, lam


def precond_apply(U, lam, mu, R):
    """P^{-1} R for the preconditioner of K + mu I built from K ~ U diag(lam) U^T."""
    R = np.asarray(R, dtype=np.float64)
    T = U.T @ R
    scale = (lam[-1] + mu) / (lam + mu)
    return U @ (scale[:, None] * T if R.ndim == 2 else scale * T) + (R - U @ T)


def pcg(X, theta, kind, b, shift=0.0, U=None, lam=None, tol=1e-10, maxit=10000, x0=None):
    """Solve (A + shift I) x = b by CG, preconditioned by the Nystrom factor if given.
    Returns (x, iterations); stops at |b - (A + shift I) x| <= tol |b| (recurrence residual)."""
    b = np.asarray(b, dtype=np.float64)
    _, _, sigma2 = gp.unpack_theta(theta, kind, np.asarray(X).shape[1])
    A = gp.a_matrix(X, theta, kind) + shift * np.eye(len(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x

    def prec(v):
        return v if U is None else precond_apply(U, lam, sigma2 + shift, v)

    z = prec(r)
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    for it in range(maxit):
        if np.linalg.norm(r) <= tol * nb:
            return x, it
        q = A @ p
        a = rz / (p @ q)
        x = x + a * p
        r = r - a * q
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit
