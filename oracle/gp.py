"""Oracle: kernel matrix, matrix-free product and quadratic-form gradients (FP64, CPU).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Definitions followed (paper section / equation):
  * Squared-exponential kernel, Section 1:   K(x,x') = alpha * exp(-|x-x'|^2 / (2 l^2)).
    ARD variant (one length-scale per coordinate, not in the paper):
        K(x,x') = alpha * exp(-1/2 sum_k (x_k - x'_k)^2 / l_k^2).
  * Kernel-plus-noise matrix, Section 2, eq. (kerdef):  A_ij = sigma^2 delta_ij + K(x_i, x_j);
    kernel-only matrix eq. (kernmat): K_ij = K(x_i, x_j).  Constant noise variance sigma^2.
  * Hyperparameter vector theta = (log alpha, log l_1 .. log l_L, log sigma^2), natural logs,
    L = 1 (isotropic) or d (ARD).
  * Quadratic-form primitive, Section 3.2.1, capacity (3): the theta-gradient of z^T A(theta) z,
    generalised here to Q = sum_c w_c u_c^T A(theta) v_c, whose derivatives are
        dQ/dlog alpha    = sum_ij K_ij S_ij
        dQ/dlog l_k      = sum_ij K_ij (x_ik - x_jk)^2 / l_k^2 S_ij     (iso: r_ij^2 / l^2)
        dQ/dlog sigma^2  = sigma^2 sum_c w_c u_c . v_c
    with S_ij = sum_c w_c u_ic v_jc.

  * Chebyshev-amplitude kernel, Section 4 (the paper's experiments):
        K(x,x') = exp(C(x)) exp(C(x')) exp(-|x-x'|^2 / (2 l^2)),
        C(x) = sum_{m_1..m_d = 0}^{N_cheb - 1} Theta_{m_1..m_d} T_{m_1}(x^1) ... T_{m_d}(x^d),
    T_m the Chebyshev polynomials of the first kind, points in the reference box [-1,1]^d.
    theta = (Theta flattened with m_1 slowest, log l, log sigma^2): N_cheb^d + 2 entries.
    Derivatives (same Q, S as above):
        dQ/dTheta_m     = sum_ij K_ij (phi_m(x_i) + phi_m(x_j)) S_ij,  phi_m = prod_k T_{m_k}(x^k)
        dQ/dlog l       = sum_ij K_ij r_ij^2 / l^2 S_ij
        dQ/dlog sigma^2 = sigma^2 sum_c w_c u_c . v_c

Everything is computed with direct coordinate differences in float64, densely, one block of
rows at a time (a block of rows of A is formed explicitly; only the row partition is a choice
made here, the arithmetic of each entry is the definition).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ISO = "iso"
ARD = "ard"
CHEB = "cheb"


def cheb_order(n_theta_total: int, d: int) -> int:
    """N_cheb from the length of a Chebyshev-kernel theta (N_cheb^d + 2 entries)."""
    m = n_theta_total - 2
    n = max(1, int(round(m ** (1.0 / d))))
    for c in (n - 1, n, n + 1):
        if c >= 1 and c ** d == m:
            return c
    raise ValueError(f"theta of length {n_theta_total} is not N_cheb^{d} + 2")


def n_theta(kind: str, d: int, n_cheb: int | None = None) -> int:
    """Number of hyperparameters: (log alpha, log l..., log sigma^2), or for the Chebyshev
    kernel (Theta (N_cheb^d), log l, log sigma^2)."""
    if kind == ISO:
        return 3
    if kind == ARD:
        return d + 2
    if kind == CHEB:
        if n_cheb is None:
            raise ValueError("the Chebyshev kernel needs n_cheb")
        return n_cheb ** d + 2
    raise ValueError(f"unknown kernel kind {kind!r}")


def unpack_theta(theta, kind: str, d: int):
    """theta -> (alpha, length-scales per coordinate (array of d), sigma^2).
    For the Chebyshev kernel alpha is 1 (the amplitude is exp(C(x)) exp(C(x')))."""
    theta = np.asarray(theta, dtype=np.float64)
    nt = n_theta(kind, d, cheb_order(theta.shape[0], d) if kind == CHEB else None)
    if theta.shape != (nt,):
        raise ValueError(f"theta has shape {theta.shape}, expected ({nt},)")
    if kind == CHEB:
        return 1.0, np.full(d, np.exp(theta[-2])), np.exp(theta[-1])
    alpha = np.exp(theta[0])
    if kind == ISO:
        ell = np.full(d, np.exp(theta[1]))
    else:
        ell = np.exp(theta[1:1 + d])
    sigma2 = np.exp(theta[-1])
    return alpha, ell, sigma2


def cheb_basis(X, n_cheb: int):
    """phi_m(x_i) = prod_k T_{m_k}(x_i^k) for every multi-index m (m_1 slowest): N x N_cheb^d."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    out = np.ones((n, 1))
    for k in range(d):
        Tk = np.polynomial.chebyshev.chebvander(X[:, k], n_cheb - 1)   # T_0..T_{N_cheb-1}
        out = (out[:, :, None] * Tk[:, None, :]).reshape(n, -1)
    return out


def cheb_log_amplitude(X, theta):
    """C(x_i) = sum_m Theta_m phi_m(x_i) (Section 4)."""
    X = np.asarray(X, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    nc = cheb_order(theta.shape[0], X.shape[1])
    return cheb_basis(X, nc) @ theta[:-2]


def _scaled_sq_diff(Xa, Xb, ell, k):
    """(x_ik - x_jk)^2 / l_k^2 for all pairs of a block: direct difference, Section 1."""
    diff = Xa[:, k][:, None] - Xb[:, k][None, :]
    return (diff * diff) / (ell[k] * ell[k])


def kernel_block(Xa, Xb, theta, kind: str):
    """Block K(x_i, x_j), i over Xa, j over Xb (Section 1; ARD generalisation)."""
    Xa = np.asarray(Xa, dtype=np.float64)
    Xb = np.asarray(Xb, dtype=np.float64)
    d = Xa.shape[1]
    alpha, ell, _ = unpack_theta(theta, kind, d)
    e = np.zeros((Xa.shape[0], Xb.shape[0]))
    for k in range(d):
        e += _scaled_sq_diff(Xa, Xb, ell, k)
    if kind == CHEB:
        amp_a = np.exp(cheb_log_amplitude(Xa, theta))
        amp_b = np.exp(cheb_log_amplitude(Xb, theta))
        return amp_a[:, None] * amp_b[None, :] * np.exp(-0.5 * e)
    return alpha * np.exp(-0.5 * e)


def a_matrix(X, theta, kind: str, no_noise: bool = False):
    """Dense A(theta) = sigma^2 I + K (eq. kerdef); K alone (eq. kernmat) if no_noise."""
    X = np.asarray(X, dtype=np.float64)
    K = kernel_block(X, X, theta, kind)
    if no_noise:
        return K
    _, _, sigma2 = unpack_theta(theta, kind, X.shape[1])
    return K + sigma2 * np.eye(X.shape[0])


def _row_blocks(rows, n_cols, max_entries=1 << 22):
    bs = max(1, min(len(rows), max_entries // max(1, n_cols)))
    return [rows[s:s + bs] for s in range(0, len(rows), bs)]


def _default_workers():
    return max(1, min(16, os.cpu_count() or 1))


def _as2d(V):
    V = np.asarray(V, dtype=np.float64)
    return (V[:, None], True) if V.ndim == 1 else (V, False)


def matvec(X, theta, kind: str, V, col_shift=None, no_noise: bool = False, rows=None,
           workers: int | None = None):
    """Rows `rows` (default: all) of (A(theta) + diag(col_shift_c)) V, column by column.

    A is eq. (kerdef) (or eq. (kernmat) with no_noise).  col_shift_c adds lambda_c I to the
    matrix applied to column c, the shifted systems of the pole expansion (Section 3.1, eq. pex).
    """
    X = np.asarray(X, dtype=np.float64)
    V, squeeze = _as2d(V)
    n, d = X.shape
    _, _, sigma2 = unpack_theta(theta, kind, d)
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    diag = np.zeros(V.shape[1]) if no_noise else np.full(V.shape[1], sigma2)
    if col_shift is not None:
        diag = diag + np.asarray(col_shift, dtype=np.float64)
    out = np.empty((len(rows), V.shape[1]))

    def work(blk_idx):
        lo = blk_idx[0]
        blk = blocks[blk_idx[1]]
        K = kernel_block(X[blk], X, theta, kind)
        out[lo:lo + len(blk)] = K @ V + V[blk] * diag[None, :]

    blocks = _row_blocks(rows, n)
    offs = np.cumsum([0] + [len(b) for b in blocks])[:-1]
    with ThreadPoolExecutor(workers or _default_workers()) as ex:
        list(ex.map(work, [(int(o), i) for i, o in enumerate(offs)]))
    return out[:, 0] if squeeze else out


def quadform_grad(X, theta, kind: str, U, V, w=None, rows=None, workers: int | None = None):
    """Q = sum_c w_c u_c^T A v_c, its theta-gradient, and the products A U, A V.

    Returns a dict with
      grad : (n_theta,)  dQ/dtheta                      (Section 3.2.1, capacity (3))
      quad : (R,)        q_c = u_c^T A v_c (unweighted)
      AU, AV : rows of A U and A V
    With `rows` given, every sum over i (the row index of u) runs over those rows only and the
    AU/AV rows returned are those rows: the full result is the sum over a partition of rows.
    """
    X = np.asarray(X, dtype=np.float64)
    U, _ = _as2d(U)
    V, _ = _as2d(V)
    n, d = X.shape
    R = U.shape[1]
    if V.shape != U.shape or U.shape[0] != n:
        raise ValueError("U and V must both be N x R")
    w = np.ones(R) if w is None else np.asarray(w, dtype=np.float64)
    alpha, ell, sigma2 = unpack_theta(theta, kind, d)
    nt = len(theta)
    if kind == CHEB:
        Phi = cheb_basis(X, cheb_order(nt, d))
        amp = np.exp(Phi @ np.asarray(theta, dtype=np.float64)[:-2])
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    blocks = _row_blocks(rows, n)
    offs = np.cumsum([0] + [len(b) for b in blocks])[:-1]
    AU = np.empty((len(rows), R))
    AV = np.empty((len(rows), R))
    partial_grad = np.zeros((len(blocks), nt))
    partial_quad = np.zeros((len(blocks), R))

    def work(bi):
        blk = blocks[bi]
        lo = int(offs[bi])
        Xb = X[blk]
        # K_ij with the per-coordinate scaled squared differences kept for the gradient.
        e = np.zeros((len(blk), n))
        for k in range(d):
            e += _scaled_sq_diff(Xb, X, ell, k)
        if kind == CHEB:
            K = amp[blk][:, None] * amp[None, :] * np.exp(-0.5 * e)
        else:
            K = alpha * np.exp(-0.5 * e)
        av = K @ V + sigma2 * V[blk]
        au = K @ U + sigma2 * U[blk]
        AV[lo:lo + len(blk)] = av
        AU[lo:lo + len(blk)] = au
        S = (U[blk] * w[None, :]) @ V.T          # S_ij = sum_c w_c u_ic v_jc
        W = K * S
        g = np.zeros(nt)
        if kind == CHEB:
            # dK_ij/dTheta_m = (phi_m(x_i) + phi_m(x_j)) K_ij, summed against S_ij
            g[:-2] = Phi[blk].T @ W.sum(axis=1) + Phi.T @ W.sum(axis=0)
            g[-2] = (W * e).sum()                 # dK/dlog l = K r^2 / l^2
        elif kind == ISO:
            g[0] = W.sum()                        # dK/dlog alpha = K
            g[1] = (W * e).sum()                  # dK/dlog l = K r^2 / l^2
        else:
            g[0] = W.sum()
            for k in range(d):
                g[1 + k] = (W * _scaled_sq_diff(Xb, X, ell, k)).sum()
        g[-1] = sigma2 * np.sum(w[None, :] * U[blk] * V[blk])   # dA/dlog sigma^2 = sigma^2 I
        partial_grad[bi] = g
        partial_quad[bi] = np.sum(U[blk] * av, axis=0)        # u_c^T (A v_c)

    with ThreadPoolExecutor(workers or _default_workers()) as ex:
        list(ex.map(work, range(len(blocks))))
    return {
        "grad": partial_grad.sum(axis=0),
        "quad": partial_quad.sum(axis=0),
        "AU": AU,
        "AV": AV,
    }


def quadform_value(X, theta, kind: str, U, V, w=None):
    """Q(theta) = sum_c w_c u_c^T A(theta) v_c by the dense matrix (small N only)."""
    U, _ = _as2d(U)
    V, _ = _as2d(V)
    w = np.ones(U.shape[1]) if w is None else np.asarray(w, dtype=np.float64)
    A = a_matrix(X, theta, kind)
    return float(np.sum(w * np.einsum("ic,ij,jc->c", U, A, V)))
