"""GPU parity of the Chebyshev-amplitude kernel (Section 4) against the FP64 oracle: products,
quadratic-form gradients (every Theta component, log l, log sigma^2), the phi refresh and a
plain-mode HMC trajectory on it.

Gradient errors are measured against sum_c |w_c| |u_c|^T |dA/dtheta_p| |v_c| (dense, here),
because components pass through zero.  Tolerances: 1e-11 (FP64), 1e-5 (FP32), 3e-3 (GP_BF16X).
"""
import numpy as np
import pytest
import torch

from oracle import gp as ogp, hmc as ohmc, poles as opoles
from paper_2412_20884_amd import gpk
from tests.gpu_util import col_rel_err, host, rounded, to_dev

pytestmark = pytest.mark.gpu
TOL = {torch.float64: 1e-11, torch.float32: 1e-5}


def _problem(n, d, nc, seed, r=3, ell=0.3, sigma2=1e-2, scale=0.3):
    g = np.random.default_rng([seed, 501])
    X = g.uniform(-1.0, 1.0, size=(n, d))
    th = np.concatenate([scale * g.standard_normal(nc ** d), [np.log(ell), np.log(sigma2)]])
    return X, th, g.standard_normal((n, r)), g.standard_normal((n, r))


def _grad_scale(X, th, U, V, w):
    """sum_c |w_c| |u_c|^T |dA/dtheta_p| |v_c| for every component, densely."""
    d = X.shape[1]
    nc = ogp.cheb_order(len(th), d)
    K = ogp.a_matrix(X, th, "cheb", no_noise=True)
    S = (np.abs(U) * np.abs(w)[None, :]) @ np.abs(V).T
    W = K * S
    Phi = np.abs(ogp.cheb_basis(X, nc))
    out = np.empty(len(th))
    out[:-2] = Phi.T @ W.sum(axis=1) + Phi.T @ W.sum(axis=0)
    r2 = np.sum((X[:, None, :] - X[None, :, :]) ** 2, axis=2) / np.exp(th[-2]) ** 2
    out[-2] = np.sum(W * r2)
    out[-1] = np.exp(th[-1]) * np.sum(np.abs(w) * np.sum(np.abs(U * V), axis=0))
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("d,nc", [(1, 2), (1, 6), (2, 3), (3, 4)])
@pytest.mark.parametrize("r", [1, 5])
def test_cheb_kmatvec(dtype, d, nc, r):
    X, th, V, _ = _problem(1000 + 37 * d + nc, d, nc, 10 * d + nc, r=r)
    X, V = rounded(X, dtype), rounded(V, dtype)
    out = gpk.kmatvec(to_dev(X, dtype), to_dev(th, torch.float64), to_dev(V, dtype), "cheb", n_cheb=nc)
    torch.cuda.synchronize()
    ref = ogp.matvec(X, th, "cheb", V)
    assert col_rel_err(host(out), ref) < TOL[dtype]


def test_cheb_kmatvec_bf16x_and_shift():
    X, th, V, _ = _problem(2100, 2, 3, 5, r=4)
    X, V = rounded(X, torch.float32), rounded(V, torch.float32)
    shift = np.array([0.0, 0.5, 2.0, 1e-3])
    out = gpk.kmatvec(to_dev(X, torch.float32), to_dev(th, torch.float64), to_dev(V, torch.float32),
                      "cheb", prec="bf16x", col_shift=to_dev(shift, torch.float64), n_cheb=3)
    torch.cuda.synchronize()
    ref = ogp.matvec(X, th, "cheb", V, col_shift=shift)
    assert col_rel_err(host(out), ref) < 3e-3


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("d,nc", [(1, 3), (2, 2), (3, 3)])
def test_cheb_quadform_grad(dtype, sym, d, nc):
    n = 1300 + d
    X, th, U, V = _problem(n, d, nc, 40 + d + nc, r=3)
    X, U, V = rounded(X, dtype), rounded(U, dtype), rounded(V, dtype)
    if sym:
        V = U
    w = np.array([-0.5, 0.5, 1.25])
    Ud = to_dev(U, dtype)
    Vd = Ud if sym else to_dev(V, dtype)
    res = gpk.quadform_grad(to_dev(X, dtype), to_dev(th, torch.float64), Ud, Vd,
                            to_dev(w, torch.float64), "cheb", want_AU=True, want_AV=True, n_cheb=nc)
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, "cheb", U, V, w)
    scale = _grad_scale(X, th, U, V, w)
    err = np.max(np.abs(host(res["grad"]) - ref["grad"]) / scale)
    assert err < TOL[dtype], (host(res["grad"]), ref["grad"])
    assert col_rel_err(host(res["AU"]), ref["AU"]) < TOL[dtype]
    assert col_rel_err(host(res["AV"]), ref["AV"]) < TOL[dtype]
    qs = np.sum(np.abs(U) * np.abs(ogp.matvec(X, th, "cheb", np.abs(V))), axis=0)
    assert np.max(np.abs(host(res["quad"]) - ref["quad"]) / qs) < TOL[dtype]


def test_cheb_quadform_bf16x():
    X, th, U, _ = _problem(2300, 2, 3, 77, r=2)
    X, U = rounded(X, torch.float32), rounded(U, torch.float32)
    w = np.array([-0.5, 0.5])
    Ud = to_dev(U, torch.float32)
    res = gpk.quadform_grad(to_dev(X, torch.float32), to_dev(th, torch.float64), Ud, Ud,
                            to_dev(w, torch.float64), "cheb", prec="bf16x", want_AU=True, n_cheb=3)
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, "cheb", U, U, w)
    assert np.max(np.abs(host(res["grad"]) - ref["grad"]) / _grad_scale(X, th, U, U, w)) < 3e-3
    assert col_rel_err(host(res["AU"]), ref["AU"]) < 3e-3


def test_cheb_constant_amplitude_equals_iso_on_gpu():
    # only Theta_0 = c: the Chebyshev path must reproduce the isotropic SE path with log alpha = 2c
    X, _, U, _ = _problem(1500, 2, 3, 9, r=2)
    th = np.zeros(11)
    th[0], th[-2], th[-1] = 0.21, np.log(0.3), np.log(1e-2)
    th_iso = np.array([0.42, np.log(0.3), np.log(1e-2)])
    Xd, Ud = to_dev(X, torch.float64), to_dev(U, torch.float64)
    rc = gpk.quadform_grad(Xd, to_dev(th, torch.float64), Ud, Ud, None, "cheb", want_AU=True, n_cheb=3)
    ri = gpk.quadform_grad(Xd, to_dev(th_iso, torch.float64), Ud, Ud, None, "iso", want_AU=True)
    torch.cuda.synchronize()
    gc, gi = host(rc["grad"]), host(ri["grad"])
    assert abs(gc[0] - 2 * gi[0]) < 1e-11 * abs(gi[0])
    assert abs(gc[-2] - gi[1]) < 1e-11 * abs(gi[1]) and abs(gc[-1] - gi[2]) < 1e-12 * abs(gi[2])
    assert col_rel_err(host(rc["AU"]), host(ri["AU"])) < 1e-12


def test_quadform_no_noise_se():
    X, _, U, _ = _problem(900, 2, 2, 12, r=2)
    th = np.array([0.3, np.log(0.25), np.log(0.05)])
    Ud = to_dev(U, torch.float64)
    res = gpk.quadform_grad(to_dev(X, torch.float64), to_dev(th, torch.float64), Ud, Ud, None, "iso",
                            want_AU=True, no_noise=True)
    torch.cuda.synchronize()
    K = ogp.a_matrix(X, th, "iso", no_noise=True)
    assert col_rel_err(host(res["AU"]), K @ U) < 1e-12
    ref = ogp.quadform_grad(X, th, "iso", U, U)
    g = host(res["grad"])
    assert g[2] == 0.0
    assert np.max(np.abs(g[:2] - ref["grad"][:2]) / np.abs(ref["grad"][:2])) < 1e-11
    np.testing.assert_allclose(host(res["quad"]), np.einsum("ic,ic->c", U, K @ U), rtol=1e-11)


def test_cheb_phi_refresh():
    X, th, _, _ = _problem(800, 2, 3, 21, r=1, sigma2=5e-2)
    xi = np.random.default_rng(5).standard_normal((800, 2))
    res = gpk.phi_refresh(to_dev(X, torch.float64), to_dev(th, torch.float64), to_dev(xi, torch.float64),
                          "cheb", tol=1e-13, maxit=5000, n_cheb=3)
    torch.cuda.synchronize()
    assert np.all(host(res["status"]) == 0)
    M = res["bounds"][1]
    assert M == pytest.approx(opoles.gershgorin_upper(X, th, "cheb") * (1 + 1e-12), rel=1e-12)
    ref = opoles.inv_sqrt_apply(X, th, "cheb", xi, M=M)
    assert col_rel_err(host(res["phi"]), ref) < 1e-9


@pytest.mark.parametrize("mode", [gpk.PLAIN, gpk.BATCHED, gpk.GRAPH])
def test_cheb_trajectory_fp64(mode):
    """The paper's verification setting (Section 4.1) scaled up: d = 1, N_cheb = 2, 2 l^2 = 1,
    sigma^2 = 0.1, here with N = 200 points on [-1, 1) and y = cos(3 x); 6 leapfrog steps."""
    n = 200
    X = (-1.0 + 2.0 * np.arange(n) / n)[:, None]
    y = np.cos(3.0 * X[:, 0])
    th = np.array([0.01, 0.01, np.log(np.sqrt(0.5)), np.log(0.1)])
    A = ogp.a_matrix(X, th, "cheb")
    xi = np.random.default_rng(3).standard_normal(n)
    phi = np.linalg.solve(np.linalg.cholesky(A).T, xi)
    pi0 = np.random.default_rng(4).standard_normal(4)
    thd = to_dev(th, torch.float64)
    pid = to_dev(pi0, torch.float64)
    xd = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    r = gpk.hmc_leapfrog(to_dev(X, torch.float64).reshape(-1, 1), to_dev(y, torch.float64),
                         to_dev(phi, torch.float64), thd, pid, xd, "cheb", [n], [0], 1, d=[1],
                         n_steps=6, dt=0.05, cg_tol=1e-12, cg_maxit=2000, mode=mode, n_cheb=2)
    torch.cuda.synchronize()
    th1, pi1 = ohmc.leapfrog(X, "cheb", y, phi, th, pi0, 0.05, 6)
    assert int(r["status"][0]) == 0
    assert np.max(np.abs(host(thd) - th1)) < 1e-8
    assert np.max(np.abs(host(pid) - pi1)) < 1e-8
    H1 = ohmc.hamiltonian(X, th1, "cheb", y, phi, pi1)
    assert abs(float(r["H1"][0]) - H1) < 1e-8 * abs(H1)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cheb_batched_chains_match_oracle_and_graph(dtype):
    """Six chains at different theta (d = 2, N_cheb = 3, N = 700, and a second instance with d = 3,
    N_cheb = 2, N = 400), 4 leapfrog steps: the persistent launch and its graph replay agree bit for
    bit, every chain follows the oracle's leapfrog (FP64 1e-8; float32 2e-4), and the plain form
    takes the same decisions."""
    C = 3
    specs = [(700, 2, 3, 41), (400, 3, 2, 42)]
    insts = []
    for n, d, nc, seed in specs:
        X, th, _, _ = _problem(n, d, nc, seed)
        X = rounded(X, dtype)
        y = rounded(np.sin(3.0 * X[:, 0]) + 0.3 * X[:, -1], dtype)
        g = np.random.default_rng([seed, 7])
        ths = [th + 0.03 * g.standard_normal(th.size) for _ in range(C)]
        phis = [rounded(np.linalg.solve(np.linalg.cholesky(ogp.a_matrix(X, t, "cheb")).T,
                                        g.standard_normal(n)), dtype) for t in ths]
        pis = [0.5 * g.standard_normal(th.size) for _ in range(C)]
        insts.append(dict(X=X, y=y, ths=ths, phis=phis, pis=pis, n=n, d=d, nc=nc))
    # both instances share N_cheb only if equal: run them as two batches of C chains each
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    for b in insts:
        n, d, nc = b["n"], b["d"], b["nc"]
        u = np.random.default_rng(n).uniform(size=C)
        out = {}
        for mode in (gpk.GRAPH, gpk.BATCHED, gpk.PLAIN):
            thd = to_dev(np.concatenate(b["ths"]), torch.float64)
            pid = to_dev(np.concatenate(b["pis"]), torch.float64)
            xd = torch.zeros(n * C, dtype=dtype, device="cuda:0")
            r = gpk.hmc_leapfrog(to_dev(b["X"], dtype).reshape(-1, 1), to_dev(b["y"], dtype),
                                 to_dev(np.concatenate(b["phis"]), dtype), thd, pid, xd, "cheb",
                                 [n], [0], C, d=[d], u=to_dev(u, torch.float64), n_steps=4,
                                 dt=0.03, cg_tol=tol, cg_maxit=4000, mode=mode, n_cheb=nc)
            torch.cuda.synchronize()
            out[mode] = {"theta": host(thd), "pi": host(pid), "H0": host(r["H0"]),
                         "H1": host(r["H1"]), "accepted": r["accepted"].cpu().numpy(),
                         "status": r["status"].cpu().numpy()}
        for key in out[gpk.GRAPH]:
            np.testing.assert_array_equal(out[gpk.GRAPH][key], out[gpk.BATCHED][key], err_msg=key)
        np.testing.assert_array_equal(out[gpk.GRAPH]["accepted"], out[gpk.PLAIN]["accepted"])
        assert np.all(out[gpk.GRAPH]["status"] == 0)
        nt = nc ** d + 2
        # float32: solves to a 1e-6 recurrence residual at condition ~1e3 give ~1e-4 in theta
        bound = 1e-8 if dtype == torch.float64 else 1e-3
        for c in range(C):
            th1, pi1 = ohmc.leapfrog(b["X"], "cheb", b["y"], b["phis"][c], b["ths"][c], b["pis"][c],
                                     0.03, 4)
            H0 = ohmc.hamiltonian(b["X"], b["ths"][c], "cheb", b["y"], b["phis"][c], b["pis"][c])
            H1 = ohmc.hamiltonian(b["X"], th1, "cheb", b["y"], b["phis"][c], pi1)
            o = out[gpk.GRAPH]
            htol = 1e-8 if dtype == torch.float64 else 1e-4
            assert abs(o["H0"][c] - H0) < htol * max(1.0, abs(H0))
            assert abs(o["H1"][c] - H1) < htol * max(1.0, abs(H1))
            got = o["theta"][c * nt:(c + 1) * nt]
            if o["accepted"][c]:
                print(f"chain {c}: |theta - oracle| {np.max(np.abs(got - th1)):.2e}")
                assert np.max(np.abs(got - th1)) < bound, (c, got - th1)
            else:
                np.testing.assert_array_equal(got, b["ths"][c])


def test_cheb_autograd_gradcheck():
    from paper_2412_20884_amd import autograd as ag

    X, th, U, _ = _problem(60, 2, 2, 31, r=2)
    Xd = to_dev(X, torch.float64)
    thd = to_dev(th, torch.float64).requires_grad_(True)
    Ud = to_dev(U, torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t, u: ag.kmatvec(Xd, t, u, "cheb", 2), (thd, Ud),
                                    eps=1e-6, atol=1e-7, rtol=1e-6)
    assert torch.autograd.gradcheck(lambda t, u: ag.quadform(Xd, t, u, None, "cheb", 2), (thd, Ud),
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


def test_cheb_plain_trajectory_two_chains_fp64():
    """Two chains of one instance in one plain-mode call (d = 2, N_cheb = 3, 3 leapfrog steps of
    0.03 with accept decisions) give exactly what each chain gives alone, and chain 1 follows the
    oracle's leapfrog."""
    n, nc, C = 300, 3, 2
    X, th, _, _ = _problem(n, 2, nc, 21)
    y = np.sin(3.0 * X[:, 0]) * np.cos(2.0 * X[:, 1])
    g = np.random.default_rng([21, 502])
    ths = [th, th + 0.05 * g.standard_normal(th.size)]
    pis = [g.standard_normal(th.size) for _ in range(C)]
    phis = [np.linalg.solve(np.linalg.cholesky(ogp.a_matrix(X, t, "cheb")).T, g.standard_normal(n))
            for t in ths]
    us = g.uniform(size=C)
    Xd, yd = to_dev(X, torch.float64).reshape(-1, 1), to_dev(y, torch.float64)

    def run(cs):
        thd = to_dev(np.concatenate([ths[c] for c in cs]), torch.float64)
        pid = to_dev(np.concatenate([pis[c] for c in cs]), torch.float64)
        xd = torch.zeros(n * len(cs), dtype=torch.float64, device="cuda:0")
        r = gpk.hmc_leapfrog(Xd, yd, to_dev(np.concatenate([phis[c] for c in cs]), torch.float64), thd,
                             pid, xd, "cheb", [n], [0], len(cs), d=[2],
                             u=to_dev(us[list(cs)], torch.float64), n_steps=3, dt=0.03, cg_tol=1e-12,
                             cg_maxit=3000, mode=gpk.PLAIN, n_cheb=nc)
        torch.cuda.synchronize()
        return {"theta": host(thd), "pi": host(pid), "x": host(xd), "H0": host(r["H0"]),
                "H1": host(r["H1"]), "accepted": r["accepted"].cpu().numpy(),
                "status": r["status"].cpu().numpy(), "cg": r["cg_iters"].cpu().numpy()}

    both = run([0, 1])
    assert np.all(both["status"] == 0)
    nt = th.size
    for c in range(C):
        one = run([c])
        for key, v in one.items():
            w = {"theta": nt, "pi": nt, "x": n}.get(key, 1)
            np.testing.assert_array_equal(both[key][c * w:(c + 1) * w], v, err_msg=f"{key} chain {c}")
    th1, pi1 = ohmc.leapfrog(X, "cheb", y, phis[1], ths[1], pis[1], 0.03, 3)
    H0 = ohmc.hamiltonian(X, ths[1], "cheb", y, phis[1], pis[1])
    H1 = ohmc.hamiltonian(X, th1, "cheb", y, phis[1], pi1)
    assert abs(float(both["H0"][1]) - H0) < 1e-8 * abs(H0)
    assert abs(float(both["H1"][1]) - H1) < 1e-8 * abs(H1)
    if both["accepted"][1]:
        assert np.max(np.abs(both["theta"][nt:] - th1)) < 1e-8
    else:
        np.testing.assert_array_equal(both["theta"][nt:], ths[1])
