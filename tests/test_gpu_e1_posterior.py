"""Statistical check of the whole sampler: the pseudofermion HMC chain targets P(theta).

The E1 problem of Section 4.1 (N = 10 points equispaced on [-1, 1), y_i = 1, sigma^2 = 0.1 held
fixed, the [-3, 3]^2 box of the paper's grid as the prior support), twice: with the paper's own
kernel there, the Chebyshev-amplitude SE kernel with N_cheb = 2 coefficients (Theta_0, Theta_1)
free and 2 l^2 = 1 fixed, and with the isotropic SE kernel's (log alpha, log l) free.
tests/golden/e1_cheb_grid_marginals.json and e1_grid_marginals.json hold the exact marginal CDFs
of P(theta) on the paper's 100^2 grid (trapezoid rule), written from the oracle's Cholesky
posterior.

500 chains (the paper's B) run Algorithm 1 on the device: per update, phi | theta is drawn
exactly (phi = L^{-T} xi with A = L L^T, on the host) or, in the third case, by the device's
Gibbs refresh of every chain at its own theta (gp_phi_refresh_chains: the pole expansion of
Section 3.1 with multi-shift CG, one graph-replayed launch), pi ~ N(0, I), and one graph-replayed
leapfrog trajectory of N_int = 3 steps of 0.4 (the paper's E1 leapfrog settings) with the
Metropolis decision on the device; the diagonal inverse mass holds the fixed hyperparameters
still (a zero entry), and a proposal outside the box is rejected by the caller (the box prior).
Chains start from the grid posterior itself (cells drawn from the joint grid density, uniform
within a cell) and run 20 updates before 200 are kept.  The empirical marginal CDFs at the grid
nodes must lie within the Dvoretzky-Kiefer-Wolfowitz radius sqrt(log(2/delta) / (2 n_eff)),
delta = 0.01, of the exact ones, with n_eff = B L / tau and tau from the Appendix C estimator on
the chain-averaged autocovariance.  A sampler that targets a different density (a wrong force
sign or factor, a wrong energy or a wrong accept rule) moves these CDFs by far more than the
radius.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import gp as ogp
from oracle import posterior, stats
from paper_2412_20884_amd import gpk
from gpu_util import DEV, host, to_dev

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _e1():
    sys.path.insert(0, GOLD)
    try:
        import make_golden
    finally:
        sys.path.remove(GOLD)
    spec, X, y, axis = make_golden.e1_data()
    gold = json.load(open(os.path.join(GOLD, "e1_grid_marginals.json")))
    gold_cheb = json.load(open(os.path.join(GOLD, "e1_cheb_grid_marginals.json")))
    return spec, X, y, axis, gold, gold_cheb, make_golden.cheb_base(spec)


@pytest.mark.parametrize("kind,refresh", [("cheb", "host"), ("iso", "host"), ("cheb", "device")])
def test_e1_marginals_within_dkw_radius(kind, refresh):
    spec, X, y, axis, gold_iso, gold_cheb, cheb_base = _e1()
    n = len(y)
    B, burn, keep = 500, 20, 200
    lo, hi = spec["grid_lo"], spec["grid_hi"]
    ls2 = np.log(spec["sigma2"])
    g = np.random.default_rng([2412, 20884])
    if kind == "cheb":
        base, n_cheb = cheb_base, spec["n_cheb"]
        inv_mass = [1.0, 1.0, 0.0, 0.0]
        cdf_gold = {0: np.asarray(gold_cheb["cdf_theta0"]), 1: np.asarray(gold_cheb["cdf_theta1"])}
    else:
        base, n_cheb = np.array([0.0, 0.0, ls2]), 0
        inv_mass = [1.0, 1.0, 0.0]
        cdf_gold = {0: np.asarray(gold_iso["cdf_log_alpha"]), 1: np.asarray(gold_iso["cdf_log_l"])}
    nt = len(base)
    # start from the grid posterior: joint cell probabilities, uniform jitter within a cell
    logp = posterior.grid_log_posterior(X, kind, y, base, (0, 1), (axis, axis))
    pc = np.exp(logp - logp.max()).ravel()
    cell = g.choice(pc.size, size=B, p=pc / pc.sum())
    h = axis[1] - axis[0]
    th0 = np.stack([axis[cell // len(axis)], axis[cell % len(axis)]], 1)
    th0 = np.clip(th0 + g.uniform(-0.5, 0.5, size=(B, 2)) * h, lo, hi)
    theta = np.concatenate([th0, np.tile(base[2:], (B, 1))], 1)

    Xd = to_dev(X, torch.float64)
    yd = to_dev(y, torch.float64)
    thd = to_dev(theta.ravel(), torch.float64)
    pid = torch.zeros(nt * B, dtype=torch.float64, device=DEV)
    phid = torch.zeros(B * n, dtype=torch.float64, device=DEV)
    xd = torch.zeros(B * n, dtype=torch.float64, device=DEV)
    ud = torch.zeros(B, dtype=torch.float64, device=DEV)
    samples = np.empty((keep, B, 2))
    acc_total = 0
    r = None  # the first call's outputs are passed back: later graph launches replay the capture
    rf = None
    xid = torch.zeros(B * n, dtype=torch.float64, device=DEV)
    for it in range(burn + keep):
        th_host = host(thd).reshape(B, nt)
        if refresh == "host":
            phi = np.empty((B, n))
            for b in range(B):
                Lc = np.linalg.cholesky(ogp.a_matrix(X, th_host[b], kind))
                phi[b] = np.linalg.solve(Lc.T, g.standard_normal(n))
            phid.copy_(torch.from_numpy(phi.ravel()))
        else:
            xid.copy_(torch.from_numpy(g.standard_normal(B * n)))
            rf = gpk.phi_refresh_chains(Xd, thd, xid, kind, [n], [0], B, tol=1e-12, maxit=500,
                                        mode=gpk.GRAPH, n_cheb=n_cheb, out=phid, outputs=rf)
            torch.cuda.synchronize()
            assert np.all(rf["status"].cpu().numpy() == 0)
        pid.copy_(torch.from_numpy(g.standard_normal(nt * B)))
        ud.copy_(torch.from_numpy(g.uniform(size=B)))
        r = gpk.hmc_leapfrog(Xd, yd, phid, thd, pid, xd, kind, [n], [0], B, u=ud, n_steps=3,
                             dt=0.4, cg_tol=1e-10, cg_maxit=200, mode=gpk.GRAPH,
                             inv_mass=inv_mass, n_cheb=n_cheb, outputs=r)
        torch.cuda.synchronize()
        st = r["status"].cpu().numpy()
        assert np.all(st == 0), np.unique(st)
        th_new = host(thd).reshape(B, nt)
        assert np.all(th_new[:, 2:] == base[2:])  # the fixed hyperparameters never move
        # the box prior: a proposal outside [-3, 3]^2 is rejected
        out = np.any((th_new[:, :2] < lo) | (th_new[:, :2] > hi), axis=1)
        th_new[out] = th_host[out]
        thd.copy_(torch.from_numpy(th_new.ravel()))
        acc = r["accepted"].cpu().numpy().astype(bool) & ~out
        if it >= burn:
            samples[it - burn] = th_new[:, :2]
            acc_total += int(acc.sum())
    rate = acc_total / (B * keep)
    report = []
    for k in (0, 1):
        tau = stats.iat_chains(samples[:, :, k].T, max_lag=100)
        n_eff = B * keep / tau
        radius = stats.dkw_radius(n_eff, delta=0.01)
        s = np.sort(samples[:, :, k].ravel())
        emp = np.searchsorted(s, axis, side="right") / s.size
        err = float(np.max(np.abs(emp - cdf_gold[k])))
        report.append((k, tau, n_eff, radius, err))
        print(f"E1 {kind} ({refresh} refresh) component {k}: tau {tau:.2f}, n_eff {n_eff:.0f}, sup CDF error {err:.4f}, "
              f"DKW radius {radius:.4f}, acceptance {rate:.3f}")
    assert 0.3 < rate < 0.98
    for k, tau, n_eff, radius, err in report:
        assert err <= radius, report
