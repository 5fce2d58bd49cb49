"""GPU parity of gp_rwm (random-walk Metropolis updates of theta given phi) against the FP64
oracle's exact-solve energies.

The proposal theta' = theta + dt * xi is formed in FP64 on both sides; the energies U_phi at theta
and theta' come from conjugate-gradient solves (tol 1e-12 in FP64, 1e-6 in FP32) on the GPU and
from Cholesky solves in the oracle.  The uniforms are placed well inside the accept / reject
regions given by the oracle's energies, so the decisions must agree exactly.
"""
import math

import numpy as np
import pytest
import torch

from oracle import hmc as ohmc
from paper_2412_20884_amd import gpk, inputs as I
from tests.gpu_util import host, rounded, to_dev
from tests.test_gpu_hmc import phi_exact

pytestmark = pytest.mark.gpu


def _batch(dtype, chains=2, specs=((500, 2), (900, 3), (333, 4)), dt=0.15):
    insts = []
    for s, (n, d) in enumerate(specs):
        p = I.ard_problem(n, d, 70 + s, sigma2=0.05)
        X, y = rounded(p["X"], dtype), rounded(p["y"], dtype)
        g = np.random.default_rng(100 + s)
        phis = [rounded(phi_exact(X, p["theta"], "ard", g.normal(size=n)), dtype) for _ in range(chains)]
        xis = [g.normal(size=d + 2) for _ in range(chains)]
        refs = [ohmc.rwm_update(X, "ard", y, phis[h], p["theta"], xis[h], dt) for h in range(chains)]
        insts.append({"X": X, "y": y, "theta": p["theta"], "phi": phis, "xi": xis, "ref": refs})
    return insts


def _run(insts, dtype, chains, dt, tol, mode, u):
    ns = [len(b["y"]) for b in insts]
    offs = np.cumsum([0] + ns[:-1])
    ds = [b["X"].shape[1] for b in insts]
    xoffs = np.cumsum([0] + [n * d for n, d in zip(ns, ds)][:-1])
    X = to_dev(np.concatenate([b["X"].ravel() for b in insts]), dtype).reshape(-1, 1)
    y = to_dev(np.concatenate([b["y"] for b in insts]), dtype)
    phi = to_dev(np.concatenate([np.concatenate(b["phi"]) for b in insts]), dtype)
    th = to_dev(np.concatenate([np.concatenate([b["theta"]] * chains) for b in insts]), torch.float64)
    xi = to_dev(np.concatenate([np.concatenate(b["xi"]) for b in insts]), torch.float64)
    xi_in = xi.clone()
    # warm starts: the solve at the start theta, which a rejected update returns unchanged
    x = to_dev(np.concatenate([np.concatenate([rounded(ohmc.solve(b["X"], b["theta"], "ard", b["y"]), dtype)] * chains)
                               for b in insts]), dtype)
    ud = None if u is None else to_dev(np.asarray(u), torch.float64)
    res = gpk.rwm(X, y, phi, th, xi, x, "ard", ns, offs, chains, d=ds, x_offsets=xoffs, u=ud,
                  dt=dt, cg_tol=tol, cg_maxit=6000, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(xi, xi_in)  # the proposal direction is left as given
    out = {k: (v.cpu().numpy() if v.dtype == torch.int32 else host(v))
           for k, v in res.items() if v is not None}
    out["theta"], out["x"] = host(th), host(x)
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("mode", [gpk.PLAIN, gpk.BATCHED, gpk.GRAPH])
def test_rwm_matches_oracle(dtype, mode):
    chains, dt = 2, 0.15
    insts = _batch(dtype, chains, dt=dt)
    # chain 0 of every instance: u at half the acceptance probability (accept); chain 1: above it
    # when the proposal is clearly uphill (reject), else again half of it
    u, expect = [], []
    for b in insts:
        for h in range(chains):
            a = min(1.0, math.exp(b["ref"][h]["U0"] - b["ref"][h]["U1"]))
            if h == 1 and a < 0.6:
                u.append(min(0.999999, 1.5 * a))
                expect.append(0)
            else:
                u.append(0.5 * a)
                expect.append(1)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    r = _run(insts, dtype, chains, dt, tol, mode, u)
    e_tol = 1e-9 if dtype == torch.float64 else 1e-4
    pos = c = xrow = 0
    for b in insts:
        nth = len(b["theta"])
        for h in range(chains):
            ref = b["ref"][h]
            assert r["status"][c] == 0
            assert r["accepted"][c] == expect[c], (c, ref["U0"], ref["U1"], u[c])
            want = ref["theta_prop"] if expect[c] else b["theta"]
            np.testing.assert_allclose(r["theta"][pos:pos + nth], want, rtol=1e-15, atol=1e-15)
            assert abs(r["U0"][c] - ref["U0"]) < e_tol * max(1.0, abs(ref["U0"]))
            assert abs(r["U1"][c] - ref["U1"]) < e_tol * max(1.0, abs(ref["U1"]))
            # x_warm returns the solve at the returned theta
            n = len(b["y"])
            xs = ohmc.solve(b["X"], r["theta"][pos:pos + nth], "ard", b["y"])
            xo = r["x"][xrow + h * n:xrow + (h + 1) * n]
            assert np.max(np.abs(xo - xs)) < (1e-7 if dtype == torch.float64 else 5e-3) * max(1.0, np.max(np.abs(xs)))
            pos += nth
            c += 1
        xrow += chains * len(b["y"])


def test_rwm_without_decision_keeps_every_proposal():
    chains, dt = 2, 0.3
    insts = _batch(torch.float64, chains, specs=((400, 3),), dt=dt)
    r = _run(insts, torch.float64, chains, dt, 1e-12, gpk.BATCHED, None)
    b = insts[0]
    nth = len(b["theta"])
    for h in range(chains):
        assert r["accepted"][h] == 1 and r["status"][h] == 0
        np.testing.assert_allclose(r["theta"][h * nth:(h + 1) * nth], b["ref"][h]["theta_prop"],
                                   rtol=1e-15, atol=1e-15)
        assert abs(r["U1"][h] - b["ref"][h]["U1"]) < 1e-9 * max(1.0, abs(b["ref"][h]["U1"]))


def test_rwm_zero_step_accepts_with_equal_energies():
    chains = 1
    insts = _batch(torch.float64, chains, specs=((300, 2),), dt=0.0)
    r = _run(insts, torch.float64, chains, 0.0, 1e-12, gpk.PLAIN, [0.999999])
    assert r["accepted"][0] == 1
    assert abs(r["U0"][0] - r["U1"][0]) < 1e-9 * max(1.0, abs(r["U0"][0]))
    np.testing.assert_array_equal(r["theta"], insts[0]["theta"])
