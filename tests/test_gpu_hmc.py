"""GPU parity of gp_hmc_leapfrog against the FP64 oracle's exact-solve trajectories.

The oracle integrates with Cholesky solves; the GPU with conjugate gradients to a relative
residual tol.  At tol 1e-12 (FP64) the solve error is below kappa * 1e-12 and the trajectories
agree to 1e-8; at the production tol 1e-6 (FP32) the agreement is looser and stated per test.
"""
import math

import numpy as np
import pytest
import torch
from scipy.linalg import cholesky, solve_triangular

from oracle import gp as ogp
from oracle import hmc as ohmc
from paper_2412_20884_amd import gpk, inputs as I
from tests.gpu_util import DEV, host, rounded, to_dev

pytestmark = pytest.mark.gpu


def phi_exact(X, th, kind, xi):
    """phi ~ N(0, A^{-1}) as L^{-T} xi with A = L L^T (any square root is exact)."""
    A = ogp.a_matrix(X, th, kind)
    L = cholesky(A, lower=True)
    return solve_triangular(L.T, xi, lower=False)


def run(insts, kind, dtype, chains, n_steps, dt, tol, mode, maxit=4000, u=None, precond=None,
        prec=None):
    """insts: list of dict(X, y, theta, phi[chains], pi[chains], x0[chains])."""
    ns = [len(b["y"]) for b in insts]
    offs = np.cumsum([0] + ns[:-1])
    ds = [b["X"].shape[1] for b in insts]
    xoffs = np.cumsum([0] + [n * d for n, d in zip(ns, ds)][:-1])
    X = np.concatenate([b["X"].ravel() for b in insts])
    y = np.concatenate([b["y"] for b in insts])
    phi = np.concatenate([np.concatenate(b["phi"]) for b in insts])
    x0 = np.concatenate([np.concatenate(b["x0"]) for b in insts])
    th = np.concatenate([np.concatenate([b["theta"]] * chains) for b in insts])
    pi = np.concatenate([np.concatenate(b["pi"]) for b in insts])
    Xd = to_dev(X, dtype).reshape(-1, 1)
    thd, pid = to_dev(th, torch.float64), to_dev(pi, torch.float64)
    xd = to_dev(x0, dtype)
    ud = None if u is None else to_dev(u, torch.float64)
    res = gpk.hmc_leapfrog(Xd, to_dev(y, dtype), to_dev(phi, dtype), thd, pid, xd, kind, ns, offs,
                           chains, d=ds, x_offsets=xoffs, u=ud, n_steps=n_steps, dt=dt,
                           cg_tol=tol, cg_maxit=maxit, mode=mode, precond=precond, prec=prec)
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if v.dtype == torch.int32 else host(v))
           for k, v in res.items() if v is not None}
    out["theta"] = host(thd)
    out["pi"] = host(pid)
    out["x"] = host(xd)
    return out


def single(X, y, th, phi, pi, x0):
    return {"X": X, "y": y, "theta": th, "phi": [phi], "pi": [pi], "x0": [x0]}


@pytest.mark.parametrize("mode", [gpk.PLAIN, gpk.BATCHED, gpk.GRAPH])
def test_small_fp64_trajectory(mode):
    w = I.small_fp64()
    X, y, th = w["X"], w["y"], w["theta"]
    phi = phi_exact(X, th, "iso", w["xi"])
    r = run([single(X, y, th, phi, w["pi"], np.zeros(len(y)))], "iso", torch.float64, 1,
            w["n_steps"], w["dt"], 1e-12, mode)
    th1, pi1 = ohmc.leapfrog(X, "iso", y, phi, th, w["pi"], w["dt"], w["n_steps"])
    assert np.max(np.abs(r["theta"] - th1)) < 1e-8, (r["theta"], th1)
    assert np.max(np.abs(r["pi"] - pi1)) < 1e-8
    H0 = ohmc.hamiltonian(X, th, "iso", y, phi, w["pi"])
    H1 = ohmc.hamiltonian(X, th1, "iso", y, phi, pi1)
    assert abs(r["H0"][0] - H0) < 1e-8 * abs(H0) and abs(r["H1"][0] - H1) < 1e-8 * abs(H1)
    assert r["status"][0] == 0 and r["accepted"][0] == 1
    np.testing.assert_allclose(r["x"], ohmc.solve(X, th1, "iso", y), rtol=0, atol=1e-7)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("mode", [gpk.PLAIN, gpk.BATCHED])
def test_batched_instances_match_oracle(dtype, mode):
    chains = 2
    specs = [(600, 2), (1000, 3), (333, 5)]
    insts = []
    for s, (n, d) in enumerate(specs):
        p = I.ard_problem(n, d, 40 + s, sigma2=0.05)
        X = rounded(p["X"], dtype)
        y = rounded(p["y"], dtype)
        g = np.random.default_rng(s)
        phis = [rounded(phi_exact(X, p["theta"], "ard", g.normal(size=n)), dtype) for _ in range(chains)]
        pis = [g.normal(size=d + 2) for _ in range(chains)]
        insts.append({"X": X, "y": y, "theta": p["theta"], "phi": phis, "pi": pis,
                      "x0": [np.zeros(n)] * chains})
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    steps, dt = 5, 0.02
    r = run(insts, "ard", dtype, chains, steps, dt, tol, mode)
    bound = 1e-8 if dtype == torch.float64 else 2e-4
    # theta / pi are packed [inst][chain][n_theta]
    pos = 0
    c = 0
    for b in insts:
        nth = len(b["theta"])
        for h in range(chains):
            th1, pi1 = ohmc.leapfrog(b["X"], "ard", b["y"], b["phi"][h], b["theta"], b["pi"][h], dt, steps)
            H1 = ohmc.hamiltonian(b["X"], th1, "ard", b["y"], b["phi"][h], pi1)
            assert np.max(np.abs(r["theta"][pos:pos + nth] - th1)) < bound
            assert np.max(np.abs(r["pi"][pos:pos + nth] - pi1)) < bound
            assert abs(r["H1"][c] - H1) < (1e-8 if dtype == torch.float64 else 1e-4) * max(1.0, abs(H1))
            assert r["status"][c] == 0
            pos += nth
            c += 1


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("mode", [gpk.PLAIN, gpk.GRAPH])
def test_wide_instances_match_oracle(dtype, mode):
    """ARD chains with d = 20 and d = 40 (padded widths 32 and 64): in plain mode their product
    jobs run in the product-only tile kernel and the gradient passes in the shared one, in graph
    mode every job in the persistent launch; length-scales in [2, 8] keep the off-diagonal
    kernel values O(0.1), so the products are not nearly diagonal."""
    chains = 2
    insts = []
    for s, (n, d) in enumerate([(520, 20), (450, 40)]):
        p = I.ard_problem(n, d, 60 + s, lo=2.0, hi=8.0, sigma2=0.05)
        X = rounded(p["X"], dtype)
        y = rounded(p["y"], dtype)
        g = np.random.default_rng(70 + s)
        phis = [rounded(phi_exact(X, p["theta"], "ard", g.normal(size=n)), dtype) for _ in range(chains)]
        pis = [0.3 * g.normal(size=d + 2) for _ in range(chains)]
        insts.append({"X": X, "y": y, "theta": p["theta"], "phi": phis, "pi": pis,
                      "x0": [np.zeros(n)] * chains})
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    steps, dt = 4, 0.02
    r = run(insts, "ard", dtype, chains, steps, dt, tol, mode)
    bound = 1e-8 if dtype == torch.float64 else 2e-4
    pos = 0
    c = 0
    for b in insts:
        nth = len(b["theta"])
        for h in range(chains):
            th1, pi1 = ohmc.leapfrog(b["X"], "ard", b["y"], b["phi"][h], b["theta"], b["pi"][h], dt, steps)
            H1 = ohmc.hamiltonian(b["X"], th1, "ard", b["y"], b["phi"][h], pi1)
            assert np.max(np.abs(r["theta"][pos:pos + nth] - th1)) < bound
            assert np.max(np.abs(r["pi"][pos:pos + nth] - pi1)) < bound
            assert abs(r["H1"][c] - H1) < (1e-8 if dtype == torch.float64 else 1e-4) * max(1.0, abs(H1))
            assert r["status"][c] == 0
            pos += nth
            c += 1


def test_accept_reject_and_restore():
    p = I.iso_problem(400, 2, 9, ell=0.3, sigma2=0.05)
    X, y, th = p["X"], p["y"], p["theta"]
    phi = phi_exact(X, th, "iso", p["xi"])
    pi0 = np.array([0.8, -0.5, 0.3])
    ref = ohmc.trajectory(X, "iso", y, phi, th, pi0, 0.05, 8)
    dH = ref["H0"] - ref["H1"]
    # u just above / below exp(H0 - H1) (capped at 1)
    a = min(1.0, math.exp(dH))
    for u, expect in ((a * 0.5, 1), (min(0.999999, a * 1.5) if a < 0.6 else None, 0)):
        if u is None:
            continue
        x0 = np.zeros(len(y))
        r = run([single(X, y, th, phi, pi0, x0)], "iso", torch.float64, 1, 8, 0.05, 1e-12,
                gpk.BATCHED, u=np.array([u]))
        assert r["accepted"][0] == expect
        if expect:
            np.testing.assert_allclose(r["theta"], ref["theta_prop"], atol=1e-8)
        else:
            np.testing.assert_array_equal(r["theta"], th)
            np.testing.assert_array_equal(r["pi"], pi0)
            np.testing.assert_array_equal(r["x"], x0)


@pytest.mark.parametrize("mode", [gpk.PLAIN, gpk.BATCHED])
def test_failure_injection(mode):
    p = I.iso_problem(300, 2, 3, ell=0.3, sigma2=0.05)
    X, y, th = p["X"], p["y"], p["theta"]
    phi = phi_exact(X, th, "iso", p["xi"])
    pi0 = np.array([0.1, 0.2, -0.1])
    # CG limited to one iteration: flagged, rejected, state restored
    r = run([single(X, y, th, phi, pi0, np.zeros(300))], "iso", torch.float64, 1, 3, 0.01, 1e-12,
            mode, maxit=1)
    assert r["status"][0] & gpk.CHAIN_CG_MAXIT and r["accepted"][0] == 0
    np.testing.assert_array_equal(r["theta"], th)
    # an absurd step drives theta out of range: non-finite, rejected
    r = run([single(X, y, th, phi, np.array([1e6, 1e6, 1e6]), np.zeros(300))], "iso", torch.float64,
            1, 3, 1e3, 1e-8, mode)
    assert r["status"][0] != 0 and r["accepted"][0] == 0
    np.testing.assert_array_equal(r["theta"], th)
    # NaN input theta
    bad = th.copy()
    bad[1] = np.nan
    r = run([single(X, y, bad, phi, pi0, np.zeros(300))], "iso", torch.float64, 1, 3, 0.01, 1e-8, mode)
    assert r["status"][0] & gpk.CHAIN_NONFINITE_THETA and r["accepted"][0] == 0


def test_reversibility_on_gpu():
    p = I.iso_problem(500, 2, 5, ell=0.3, sigma2=0.05)
    X, y, th = p["X"], p["y"], p["theta"]
    phi = phi_exact(X, th, "iso", p["xi"])
    pi0 = np.array([0.4, -0.3, 0.2])
    r1 = run([single(X, y, th, phi, pi0, np.zeros(500))], "iso", torch.float64, 1, 10, 0.03, 1e-13, gpk.BATCHED)
    r2 = run([single(X, y, r1["theta"], phi, -r1["pi"], r1["x"])], "iso", torch.float64, 1, 10, 0.03, 1e-13,
             gpk.BATCHED)
    np.testing.assert_allclose(r2["theta"], th, atol=1e-9)
    np.testing.assert_allclose(-r2["pi"], pi0, atol=1e-9)


def test_graph_replays_match_batched_bitwise():
    p = I.ard_problem(700, 3, 8, sigma2=0.05)
    X, y, th = rounded(p["X"], torch.float32), rounded(p["y"], torch.float32), p["theta"]
    phi = rounded(phi_exact(X, th, "ard", p["xi"]), torch.float32)
    pi0 = np.array([0.3, -0.2, 0.1, 0.05, -0.1])
    outs = {}
    for mode in (gpk.BATCHED, gpk.GRAPH):
        Xd = to_dev(X, torch.float32)
        yd, phid = to_dev(y, torch.float32), to_dev(phi, torch.float32)
        thd, pid = to_dev(th, torch.float64), to_dev(pi0, torch.float64)
        xd = torch.zeros(700, dtype=torch.float32, device=DEV)
        hist = []
        for rep in range(3):
            res = gpk.hmc_leapfrog(Xd, yd, phid, thd, pid, xd, "ard", [700], [0], 1, n_steps=4,
                                   dt=0.02, cg_tol=1e-6, mode=mode)
            torch.cuda.synchronize()
            hist.append((host(thd).copy(), host(pid).copy(), host(res["H1"]).copy()))
            pid.neg_()   # a different momentum for the next replay
        outs[mode] = hist
    for a, b in zip(outs[gpk.BATCHED], outs[gpk.GRAPH]):
        for x, z in zip(a, b):
            np.testing.assert_array_equal(x, z)


@pytest.mark.parametrize("kind,specs", [("ard", [(1500, 20), (777, 40)]), ("iso", [(1111, 3)])])
def test_bf16x_trajectories_all_modes(kind, specs):
    """GP_BF16X trajectories on the matrix-core tiles (cross term in bfloat16 hi/lo, everything
    else in float) in the three modes, against the FP64 oracle, to the precision's 3e-3 budget:
    the displacements theta_1 - theta_0 and pi_1 - pi_0 of 4 steps, and both energies, within
    3e-3 of their size (the kernel values' relative error, a few eps32 |x~|^2, reaches the solves
    amplified by the condition number: ~1e-5 in the force at d = 20, ~5e-4 for the isotropic
    d = 3 problem, whose near pairs make A ill-conditioned).  Instances of different d
    (cross-term widths 32 and 64) and ragged N (not multiples of the 32-column tiles, the 64-row
    stage blocks or the 128-row product blocks) share one persistent launch; its graph replay
    equals it bit for bit, and the plain mode runs the same tiles one job at a time."""
    chains = 2
    insts = []
    for s, (n, d) in enumerate(specs):
        if kind == "ard":
            p = I.ard_problem(n, d, 23 + s, lo=0.5, hi=4.0, sigma2=0.05)
        else:
            p = I.iso_problem(n, d, 23 + s, ell=0.3, sigma2=0.05)
        X, y = rounded(p["X"], torch.float32), rounded(p["y"], torch.float32)
        g = np.random.default_rng(100 + s)
        phis = [rounded(phi_exact(X, p["theta"], kind, g.normal(size=n)), torch.float32)
                for _ in range(chains)]
        pis = [g.normal(size=len(p["theta"])) * 0.5 for _ in range(chains)]
        insts.append({"X": X, "y": y, "theta": p["theta"], "phi": phis, "pi": pis,
                      "x0": [np.zeros(n)] * chains})
    steps, dt = 4, 0.02
    outs = {mode: run(insts, kind, torch.float32, chains, steps, dt, 1e-6, mode, prec="bf16x")
            for mode in (gpk.PLAIN, gpk.BATCHED, gpk.GRAPH)}
    for key in ("theta", "pi", "H0", "H1", "x", "accepted", "status"):
        np.testing.assert_array_equal(outs[gpk.BATCHED][key], outs[gpk.GRAPH][key])
    for key in ("theta", "pi"):
        np.testing.assert_allclose(outs[gpk.PLAIN][key], outs[gpk.BATCHED][key], rtol=0, atol=1e-6)
    r = outs[gpk.BATCHED]
    pos = c = 0
    for b in insts:
        nth = len(b["theta"])
        for h in range(chains):
            th1, pi1 = ohmc.leapfrog(b["X"], kind, b["y"], b["phi"][h], b["theta"], b["pi"][h], dt,
                                     steps)
            H0 = ohmc.hamiltonian(b["X"], b["theta"], kind, b["y"], b["phi"][h], b["pi"][h])
            H1 = ohmc.hamiltonian(b["X"], th1, kind, b["y"], b["phi"][h], pi1)
            assert r["status"][c] == 0
            dth = np.max(np.abs(th1 - b["theta"]))
            dpi = np.max(np.abs(pi1 - b["pi"][h]))
            assert np.max(np.abs(r["theta"][pos:pos + nth] - th1)) < 3e-3 * dth
            assert np.max(np.abs(r["pi"][pos:pos + nth] - pi1)) < 3e-3 * dpi
            assert abs(r["H0"][c] - H0) < 3e-3 * abs(H0)
            assert abs(r["H1"][c] - H1) < 3e-3 * abs(H1)
            pos += nth
            c += 1


def test_bf16x_rejects_cheb_and_precond():
    """GP_BF16X trajectories take the SE kernels without a preconditioner."""
    p = I.ard_problem(300, 3, 5, sigma2=0.05)
    Xd = to_dev(p["X"], torch.float32)
    yd = to_dev(p["y"], torch.float32)
    phid = to_dev(p["xi"], torch.float32)
    thd = to_dev(p["theta"], torch.float64)
    pid = torch.zeros(5, dtype=torch.float64, device=DEV)
    xd = torch.zeros(300, dtype=torch.float32, device=DEV)
    U = torch.zeros(300, 4, dtype=torch.float32, device=DEV)
    lam = torch.ones(1, 4, dtype=torch.float64, device=DEV)
    with pytest.raises(gpk.GpkError):
        gpk.hmc_leapfrog(Xd, yd, phid, thd, pid, xd, "ard", [300], [0], 1, n_steps=1,
                         mode=gpk.BATCHED, prec="bf16x", precond=(U, lam))
