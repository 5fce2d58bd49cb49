"""Batched Gibbs refresh phi_c = A(theta_c)^{-1/2} xi_c (Section 3.1, eq. pex; Appendix A, eq.
msqdisc) through gp_phi_refresh_chains: chains of several instances, each at its own theta, in
the plain, batched (one persistent launch) and graph modes, against the oracle's pole expansion
with exact (Cholesky) shifted solves.

Tolerances follow the single-theta refresh (test_gpu_phi.py): each shifted system stops at
relative residual `tol`, which bounds its relative error by (M / m) tol; in float32 the solves
reach (M / m) eps32.  The oracle uses the m and M the call reports, so the expansion's own error
cancels.  The device forms the weights and shifts itself (double-precision AGM), the oracle with
scipy's elliptic functions.
"""
import numpy as np
import pytest
import torch

from oracle import poles as opoles
from paper_2412_20884_amd import gpk, inputs as I
from tests.gpu_util import host, rounded, to_dev

pytestmark = pytest.mark.gpu
EPS32 = 2.0 ** -24


def _col_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _batch(kind, ns, ds, chains, seed, sigma2s, n_cheb=0):
    """Instances of ns[b] points in ds[b] dimensions, chains per instance at different theta
    (length-scales and sigma^2 varied per chain), xi ~ N(0, I) per chain."""
    g = np.random.default_rng([seed, 77])
    Xs, ths, xis = [], [], []
    for b, (n, d) in enumerate(zip(ns, ds)):
        Xs.append(g.uniform(0.0, 1.0, size=(n, d)) if kind != "cheb" else g.uniform(-1, 1, (n, d)))
        for h in range(chains):
            s2 = sigma2s[(b * chains + h) % len(sigma2s)]
            if kind == "iso":
                th = I.theta_iso(np.exp(0.3 * g.standard_normal()), 0.15 * np.exp(0.3 * g.standard_normal()), s2)
            elif kind == "ard":
                th = np.concatenate([[0.2 * g.standard_normal()], np.log(g.uniform(0.1, 0.6, d)), [np.log(s2)]])
            else:
                th = np.concatenate([0.3 * g.standard_normal(n_cheb ** d), [np.log(0.3), np.log(s2)]])
            ths.append(th)
            xis.append(g.standard_normal(n))
    offs = np.cumsum([0] + list(ns[:-1]))
    return Xs, ths, xis, [int(o) for o in offs]


def _pack(Xs, ths, xis, ns, chains, dtype):
    X = np.concatenate([x.ravel() for x in Xs])
    xi = np.concatenate(xis)  # chain h of instance b at chains * off_b + h * n_b: instance-major
    return (to_dev(rounded(X, dtype), dtype), to_dev(np.concatenate(ths), torch.float64),
            to_dev(rounded(xi, dtype), dtype))


def _xoffs(Xs):
    """Element offsets of the instances' coordinates (their dimensions differ)."""
    return [int(o) for o in np.cumsum([0] + [x.size for x in Xs[:-1]])]


def _run(Xs, ths, xis, ns, ds, offs, chains, kind, dtype, mode, **kw):
    X, th, xi = _pack(Xs, ths, xis, ns, chains, dtype)
    res = gpk.phi_refresh_chains(X.view(-1, 1), th, xi, kind, ns, offs, chains, d=ds,
                                 x_offsets=_xoffs(Xs), mode=mode, **kw)
    torch.cuda.synchronize()
    return res, xi


def _check_vs_oracle(res, Xs, ths, xis, ns, chains, kind, dtype, bound_of):
    phi = host(res["phi"])
    bounds = host(res["bounds"]).reshape(-1, 2)
    st = host(res["status"])
    o = 0
    worst = 0.0
    for b, n in enumerate(ns):
        for h in range(chains):
            c = b * chains + h
            th = ths[c]
            m, M = bounds[c]
            assert st[c] == 0, f"chain {c} status {st[c]}"
            assert m == pytest.approx(np.exp(th[-1]), rel=1e-15)
            Xr = rounded(Xs[b], dtype)
            ref = opoles.inv_sqrt_apply(Xr, th, kind, rounded(xis[c], dtype), M=M)
            err = _col_err(phi[o:o + n], ref)
            worst = max(worst, err / bound_of(m, M))
            assert err < bound_of(m, M), f"chain {c}: rel err {err:.3e}, bound {bound_of(m, M):.3e}"
            o += n
    return worst


@pytest.mark.parametrize("mode", [gpk.PLAIN, gpk.BATCHED, gpk.GRAPH])
def test_chains_fp64_vs_oracle(mode):
    """Three instances (n = 300 at d = 2, 517 at d = 3 with a ragged last tile, and n = 1) x 3
    chains, every chain at its own theta; the Gershgorin bound formed on the device."""
    ns, ds, C = [300, 517, 1], [2, 3, 2], 3
    Xs, ths, xis, offs = _batch("ard", ns, ds, C, 5, [1e-2, 3e-2, 0.1])
    res, _ = _run(Xs, ths, xis, ns, ds, offs, C, "ard", torch.float64, mode, tol=1e-13, maxit=5000)
    bounds = host(res["bounds"]).reshape(-1, 2)
    for b, n in enumerate(ns):
        for h in range(C):
            c = b * C + h
            M_ref = opoles.gershgorin_upper(Xs[b], ths[c], "ard")
            assert bounds[c, 1] == pytest.approx(M_ref * (1 + 1e-12), rel=1e-12)
    _check_vs_oracle(res, Xs, ths, xis, ns, C, "ard", torch.float64,
                     lambda m, M: 1e-12 + 10 * (M / m) * 1e-13)


def test_chains_modes_agree_and_graph_replays():
    """Batched and graph modes run the same jobs in the same order: bitwise equal, also on a
    second graph replay with new xi; plain mode (column-split products) agrees to rounding."""
    ns, ds, C = [400, 250], [3, 3], 4
    Xs, ths, xis, offs = _batch("iso", ns, ds, C, 9, [1e-2, 5e-2])
    kw = dict(tol=1e-12, maxit=4000)
    a, _ = _run(Xs, ths, xis, ns, ds, offs, C, "iso", torch.float64, gpk.BATCHED, **kw)
    X, th, xi = _pack(Xs, ths, xis, ns, C, torch.float64)
    g1 = gpk.phi_refresh_chains(X.view(-1, 1), th, xi, "iso", ns, offs, C, d=ds, x_offsets=_xoffs(Xs),
                                mode=gpk.GRAPH, **kw)
    torch.cuda.synchronize()
    p1 = host(g1["phi"]).copy()
    xi.copy_(torch.flip(xi, [0]))  # new right-hand sides, same buffers: a replay
    g2 = gpk.phi_refresh_chains(X.view(-1, 1), th, xi, "iso", ns, offs, C, d=ds, x_offsets=_xoffs(Xs),
                                mode=gpk.GRAPH, outputs=g1, **kw)
    torch.cuda.synchronize()
    p2 = host(g2["phi"]).copy()
    xi.copy_(torch.flip(xi, [0]))
    g3 = gpk.phi_refresh_chains(X.view(-1, 1), th, xi, "iso", ns, offs, C, d=ds, x_offsets=_xoffs(Xs),
                                mode=gpk.GRAPH, outputs=g1, **kw)
    pl = gpk.phi_refresh_chains(X.view(-1, 1), th, xi, "iso", ns, offs, C, d=ds, x_offsets=_xoffs(Xs),
                                mode=gpk.PLAIN, **kw)
    torch.cuda.synchronize()
    pa = host(a["phi"])
    assert np.array_equal(pa, p1)
    assert np.array_equal(pa, host(g3["phi"]))
    assert np.array_equal(host(a["iters"]), host(g3["iters"]))
    assert not np.array_equal(p1, p2)
    assert _col_err(host(pl["phi"]), pa) < 1e-10
    # the flipped right-hand sides against the oracle too
    xf = host(torch.flip(xi, [0]))
    o = 0
    bounds = host(g2["bounds"]).reshape(-1, 2)
    for b, n in enumerate(ns):
        for h in range(C):
            c = b * C + h
            ref = opoles.inv_sqrt_apply(Xs[b], ths[c], "iso", xf[o:o + n], M=bounds[c, 1])
            assert _col_err(p2[o:o + n], ref) < 1e-12 + 10 * (bounds[c, 1] / bounds[c, 0]) * 1e-12
            o += n


def test_chains_match_single_theta_refresh():
    """Every chain equals gp_phi_refresh at that chain's theta (same m, M; different product
    kernels, so to rounding)."""
    ns, ds, C = [600], [4], 3
    Xs, ths, xis, offs = _batch("ard", ns, ds, C, 13, [2e-2])
    res, _ = _run(Xs, ths, xis, ns, ds, offs, C, "ard", torch.float64, gpk.BATCHED, tol=1e-12,
                  maxit=4000)
    phi = host(res["phi"])
    bounds = host(res["bounds"]).reshape(-1, 2)
    Xd = to_dev(Xs[0], torch.float64)
    for h in range(C):
        one = gpk.phi_refresh(Xd, to_dev(ths[h], torch.float64), to_dev(xis[h], torch.float64), "ard",
                              tol=1e-12, maxit=4000, lambda_max=bounds[h, 1])
        torch.cuda.synchronize()
        assert _col_err(phi[h * 600:(h + 1) * 600], host(one["phi"]).ravel()) < 1e-10
        # the same recurrence; in finite precision the two products' rounding steers the Krylov
        # iterates apart over hundreds of iterations, so the counts agree to a few percent
        it_b, it_1 = int(host(res["iters"])[h]), int(host(one["iters"])[0])
        assert abs(it_b - it_1) <= max(2, 0.05 * it_1)


def test_chains_caller_bound_zero_xi_inplace_maxit_and_nonfinite():
    ns, ds, C = [350, 200], [2, 2], 2
    Xs, ths, xis, offs = _batch("iso", ns, ds, C, 21, [1e-2])
    xis[1] = np.zeros(ns[0])          # instance 0, chain 1: phi = 0 at once
    ths[2] = ths[2].copy()
    ths[2][-1] = np.nan               # instance 1, chain 0: non-finite sigma^2
    M = 1.05 * max(opoles.gershgorin_upper(Xs[b], ths[b * C + h], "iso")
                   for b in range(2) for h in range(C) if b * C + h != 2)
    X, th, xi = _pack(Xs, ths, xis, ns, C, torch.float64)
    res = gpk.phi_refresh_chains(X.view(-1, 1), th, xi, "iso", ns, offs, C, d=ds, x_offsets=_xoffs(Xs),
                                 mode=gpk.BATCHED, tol=1e-12, maxit=4000, lambda_max=M, out=xi)
    torch.cuda.synchronize()
    st, it = host(res["status"]), host(res["iters"])
    bounds = host(res["bounds"]).reshape(-1, 2)
    phi = host(xi)
    assert st[2] == gpk.PHI_NONFINITE
    assert st[1] == 0 and it[1] == 0 and np.all(phi[ns[0]:2 * ns[0]] == 0.0)
    for c in (0, 3):
        assert st[c] == 0 and bounds[c, 1] == M
    o = {0: 0, 3: 2 * ns[0] + ns[1]}
    for c, b, n in ((0, 0, ns[0]), (3, 1, ns[1])):
        ref = opoles.inv_sqrt_apply(Xs[b], ths[c], "iso", xis[c], M=M)
        assert _col_err(phi[o[c]:o[c] + n], ref) < 1e-12 + 10 * (M / bounds[c, 0]) * 1e-13
    # an iteration limit below convergence
    X, th, xi = _pack(Xs, ths, xis, ns, C, torch.float64)
    lim = gpk.phi_refresh_chains(X.view(-1, 1), th, xi, "iso", ns, offs, C, d=ds, x_offsets=_xoffs(Xs),
                                 mode=gpk.GRAPH, tol=1e-13, maxit=3)
    torch.cuda.synchronize()
    st, it = host(lim["status"]), host(lim["iters"])
    for c in (0, 3):
        assert st[c] == gpk.PHI_CG_MAXIT and it[c] == 3


@pytest.mark.parametrize("kind,ds,prec", [("iso", [3, 3], None), ("ard", [8, 5], None),
                                          ("ard", [40, 24], "bf16x"), ("iso", [3, 2], "bf16x")])
def test_chains_float32(kind, ds, prec):
    ns, C = [900, 1300], 3
    Xs, ths, xis, offs = _batch(kind, ns, ds, C, 31 + ds[0], [0.1, 0.05])
    res, _ = _run(Xs, ths, xis, ns, ds, offs, C, kind, torch.float32, gpk.GRAPH, prec=prec, tol=1e-6,
                  maxit=3000)

    def bound_of(m, M, b=None):
        return 10 * (M / m) * ent

    ent = EPS32
    if prec == "bf16x":
        # the norm expansion's absolute error of a few eps32 max |x~|^2 per squared distance
        mx = 0.0
        for b in range(2):
            Xr = rounded(Xs[b], torch.float32)
            for h in range(C):
                th = ths[b * C + h]
                ell = np.exp(th[1:-1]) if kind == "ard" else np.exp(th[1])
                xt = (Xr - Xr.mean(axis=0)) * np.sqrt(np.log2(np.e) / 2) / ell
                mx = max(mx, np.max(np.sum(xt * xt, axis=1)))
        ent = 8 * EPS32 * mx * np.log(2) + EPS32
    worst = _check_vs_oracle(res, Xs, ths, xis, ns, C, kind, torch.float32, bound_of)
    print(f"phi chains {kind} d={ds} prec={prec}: worst err / bound {worst:.3e}, "
          f"iters {host(res['iters'])}")


def test_chains_cheb_fp64():
    ns, ds, C, nc = [500, 300], [2, 2], 2, 3
    Xs, ths, xis, offs = _batch("cheb", ns, ds, C, 41, [5e-2, 2e-2], n_cheb=nc)
    res, _ = _run(Xs, ths, xis, ns, ds, offs, C, "cheb", torch.float64, gpk.GRAPH, tol=1e-13,
                  maxit=5000, n_cheb=nc)
    _check_vs_oracle(res, Xs, ths, xis, ns, C, "cheb", torch.float64,
                     lambda m, M: 1e-11 + 10 * (M / m) * 1e-13)


def test_chains_rejects_preconditioner_and_bad_poles():
    X = torch.zeros(20, dtype=torch.float64, device="cuda:0")
    th = to_dev(I.theta_iso(1.0, 0.2, 1e-2), torch.float64)
    xi = torch.zeros(10, dtype=torch.float64, device="cuda:0")
    with pytest.raises(gpk.GpkError):
        gpk.phi_refresh_chains(X.view(-1, 1), th, xi, "iso", [10], [0], 1, d=[2], n_poles=65)
    with pytest.raises(gpk.GpkError):
        gpk.phi_refresh_chains(X.view(-1, 1), th, xi, "iso", [10], [0], 1, d=[2], tol=0.0)
