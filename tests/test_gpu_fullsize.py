"""Parity at the full sizes of the workloads, in the launch configuration the benchmark times.

The oracle computes sampled rows one by one (all N columns each); sums over all N^2 pairs are
checked through identities that hold at any size, and the theta-gradient element by element on
a row sample (the left operand zeroed outside it, so the gradient is the oracle's
row-restricted one).  The batched trajectories are checked for exact agreement between the
graph replay and the persistent launch, and against the plain single-chain form.  The cheb2d
workload (N = 3000, FP64) is small enough for the oracle's dense Cholesky path at full size.
"""
import numpy as np
import pytest
import torch

from oracle import gp as ogp
from oracle import hmc as ohmc
from oracle import poles as opoles
from paper_2412_20884_amd import gpk, inputs as I
from tests.gpu_util import DEV, comp_rel_err, grad_rel_err, host, rounded, to_dev

pytestmark = pytest.mark.gpu


def _rows_rel(out, ref):
    """max over columns of |out - ref|_2 / |ref|_2 on the sampled rows."""
    return float(np.max(np.linalg.norm(out - ref, axis=0) / np.linalg.norm(ref, axis=0)))


def test_large3_full_size_tuned():
    """N = 2^20, d = 3 isotropic, R = 32: the fused A Z + q + grad pass as the benchmark runs it."""
    w = I.large3()
    n, r = w["X"].shape[0], w["Z"].shape[1]
    X = rounded(w["X"], torch.float32)
    Z = rounded(w["Z"], torch.float32)
    th = w["theta"]
    gpk.tune("iso", 3, n, r, torch.float32, with_grad=True)
    Xd, Zd = to_dev(X, torch.float32), to_dev(Z, torch.float32)
    thd = to_dev(th, torch.float64)
    ws = torch.empty(gpk.workspace_size(gpk.make_kernel("iso", Xd), n, r), dtype=torch.uint8, device=DEV)
    res = gpk.quadform_grad(Xd, thd, Zd, Zd, None, "iso", want_AU=True, ws=ws)
    torch.cuda.synchronize()
    # 64 rows: 16 at random, the 24 points nearest a face and the 24 nearest a corner of the
    # unit cube (the rows whose sums are most one-sided)
    face = np.min(np.minimum(X, 1.0 - X), axis=1)
    corner = np.max(np.minimum(X, 1.0 - X), axis=1)
    rows = np.unique(np.concatenate([np.random.default_rng(5).choice(n, 16, replace=False),
                                     np.argsort(face)[:24], np.argsort(corner)[:24]]))
    ref = ogp.matvec(X, th, "iso", Z, rows=rows)
    absref = ogp.matvec(X, th, "iso", np.abs(Z), rows=rows)
    got = host(res["AU"])[rows]
    assert _rows_rel(got, ref) < 1e-5
    assert comp_rel_err(got, ref, absref) < 1e-5
    # sum_c q_c = dQ/dlog alpha + sigma^2 |Z|^2 and dQ/dlog sigma^2 = sigma^2 |Z|^2
    s2 = float(np.exp(th[2]))
    zz = float(np.sum(Z * Z))
    g, q = host(res["grad"]), host(res["quad"])
    assert abs(g[0] - (q.sum() - s2 * zz)) < 1e-5 * abs(g[0])
    assert abs(g[2] - s2 * zz) < 1e-12 * abs(g[2])
    # theta-gradient element by element on 16 rows: Z zeroed outside them on the left
    rows = np.sort(np.random.default_rng(6).choice(n, 16, replace=False))
    Zm = np.zeros_like(Z)
    Zm[rows] = Z[rows]
    res2 = gpk.quadform_grad(Xd, thd, to_dev(Zm, torch.float32), Zd, None, "iso", ws=ws)
    torch.cuda.synchronize()
    ref_g = ogp.quadform_grad(X, th, "iso", Zm, Z, rows=rows)["grad"]
    scale = ogp.quadform_grad(X, th, "iso", np.abs(Zm), np.abs(Z), rows=rows)["grad"]
    assert grad_rel_err(host(res2["grad"]), ref_g, scale) < 1e-5


def test_ard64_full_size_bf16x():
    """N = 262,144, d = 64 ARD in GP_BF16X: product rows and the force pass's row-restricted
    gradient (w = (-1/2, +1/2)) within the bfloat16 cross-term budget of 3e-3."""
    w = I.ard64()
    n = w["X"].shape[0]
    X = rounded(w["X"], torch.float32)
    th = w["theta"]
    V = rounded(w["xi"][:2].T, torch.float32)
    Xd, thd, Vd = to_dev(X, torch.float32), to_dev(th, torch.float64), to_dev(V, torch.float32)
    out = gpk.kmatvec(Xd, thd, Vd, "ard", prec="bf16x")
    torch.cuda.synchronize()
    rows = np.random.default_rng(7).choice(n, 8, replace=False)
    ref = ogp.matvec(X, th, "ard", V, rows=rows)
    o = host(out)[rows]
    assert _rows_rel(o, ref) < 3e-3
    # the off-diagonal part (K - alpha I) V against its own norm: at d = 64 A is close to
    # (alpha + sigma^2) I, so the whole product alone would meet the budget trivially
    diag = np.exp(th[0]) + np.exp(th[-1])
    od_o, od_r = o - diag * V[rows], ref - diag * V[rows]
    od_err = float(np.max(np.linalg.norm(od_o - od_r, axis=0) / np.linalg.norm(od_r, axis=0)))
    print(f"ard64 off-diagonal part: relative error {od_err:.2e}, norm ratio to the column "
          f"{float(np.min(np.linalg.norm(od_r, axis=0) / np.linalg.norm(ref, axis=0))):.1e}")
    assert od_err < 3e-3
    rows = np.sort(np.random.default_rng(8).choice(n, 8, replace=False))
    Vm = np.zeros_like(V)
    Vm[rows] = V[rows]
    wts = np.array([-0.5, 0.5])
    res = gpk.quadform_grad(Xd, thd, to_dev(Vm, torch.float32), Vd, to_dev(wts, torch.float64), "ard",
                            prec="bf16x")
    torch.cuda.synchronize()
    ref_g = ogp.quadform_grad(X, th, "ard", Vm, V, w=wts, rows=rows)["grad"]
    scale = ogp.quadform_grad(X, th, "ard", np.abs(Vm), np.abs(V), rows=rows)["grad"]
    assert grad_rel_err(host(res["grad"]), ref_g, scale) < 3e-3


def test_batched_largest_instances_full_size():
    """The largest instance of each dimension of the batched workload (N_b up to 32,768):
    sampled rows of A [y | xi_0] in FP32."""
    wl = I.batched()
    for d in (4, 8, 16):
        b = max((b for b in wl["instances"] if b["X"].shape[1] == d), key=lambda b: b["X"].shape[0])
        n = b["X"].shape[0]
        X = rounded(b["X"], torch.float32)
        V = rounded(np.stack([b["y"], b["xi"][0]], axis=1), torch.float32)
        out = gpk.kmatvec(to_dev(X, torch.float32), to_dev(b["theta"], torch.float64),
                          to_dev(V, torch.float32), "ard")
        torch.cuda.synchronize()
        rows = np.random.default_rng(9 + d).choice(n, 16, replace=False)
        ref = ogp.matvec(X, b["theta"], "ard", V, rows=rows)
        assert _rows_rel(host(out)[rows], ref) < 1e-5, (d, n)
        absref = ogp.matvec(X, b["theta"], "ard", np.abs(V), rows=rows)
        assert comp_rel_err(host(out)[rows], ref, absref) < 1e-5, (d, n)


def test_batched_trajectories_graph_persistent_plain():
    """Every 16th instance of the batched workload (real N_b and d_b), 8 chains, 20 leapfrog
    steps of dt 1e-3 (the benchmark's leapfrog leg): the graph replay equals the persistent
    launch exactly; the plain single-chain form agrees to float32 summation order."""
    wl = I.batched()
    C = wl["chains"]
    inst = wl["instances"][::16]
    ns = [b["X"].shape[0] for b in inst]
    ds = [b["X"].shape[1] for b in inst]
    offs = np.cumsum([0] + ns[:-1])
    xoffs = np.cumsum([0] + [a * b for a, b in zip(ns, ds)][:-1])
    X = to_dev(np.concatenate([b["X"].ravel() for b in inst]), torch.float32)[:, None]
    y = to_dev(np.concatenate([b["y"] for b in inst]), torch.float32)
    phi = torch.empty(sum(ns) * C, dtype=torch.float32, device=DEV)
    for bi, b in enumerate(inst):
        Xb = X[xoffs[bi]:xoffs[bi] + ns[bi] * ds[bi]].view(ns[bi], ds[bi])
        r = gpk.phi_refresh(Xb, to_dev(b["theta"], torch.float64), to_dev(b["xi"].T, torch.float32), "ard",
                            tol=1e-6, maxit=3000)
        assert np.all(r["status"].cpu().numpy() == 0)
        phi[C * offs[bi]:C * (offs[bi] + ns[bi])] = r["phi"].t().contiguous().view(-1)
    th0 = np.concatenate([np.tile(b["theta"], C) for b in inst])
    pi0 = np.concatenate([b["pi"].ravel() for b in inst])
    u = to_dev(np.concatenate([b["u"] for b in inst]), torch.float64)
    out = {}
    for mode in (gpk.GRAPH, gpk.BATCHED, gpk.PLAIN):
        th = to_dev(th0, torch.float64)
        pi = to_dev(pi0, torch.float64)
        x = torch.zeros(sum(ns) * C, dtype=torch.float32, device=DEV)
        res = gpk.hmc_leapfrog(X, y, phi, th, pi, x, "ard", ns, offs, C, d=ds, x_offsets=xoffs, u=u,
                               n_steps=wl["n_steps"], dt=wl["dt"], cg_tol=1e-6, cg_maxit=2000, mode=mode)
        torch.cuda.synchronize()
        out[mode] = {"theta": host(th), "pi": host(pi), "x": host(x), "H0": host(res["H0"]),
                     "H1": host(res["H1"]), "accepted": res["accepted"].cpu().numpy(),
                     "status": res["status"].cpu().numpy(), "cg": res["cg_iters"].cpu().numpy()}
    g, b, p = out[gpk.GRAPH], out[gpk.BATCHED], out[gpk.PLAIN]
    assert np.all(g["status"] == 0) and np.all(p["status"] == 0)
    for key in g:
        np.testing.assert_array_equal(g[key], b[key], err_msg=key)
    np.testing.assert_array_equal(g["accepted"], p["accepted"])
    assert np.max(np.abs(g["theta"] - p["theta"])) < 1e-5
    # the energies differ by float32 summation order only
    assert np.all(np.abs(g["H1"] - g["H0"] - (p["H1"] - p["H0"])) <= 2e-6 * np.abs(p["H0"]) + 1e-3)
    assert np.all(np.abs(g["cg"] - p["cg"]) <= 0.02 * p["cg"] + 2)


def test_batched_refresh_one_launch_full_size():
    """The benchmark's one-launch refresh: every chain of every 16th instance of the batched
    workload (N_b = 7018, 19409, 11616, 6050; 8 chains each, each its own system) in one
    batched-mode gp_phi_refresh_chains launch, FP32, tolerance 1e-6.  The smallest instance's 8
    chains against the oracle's pole expansion (Cholesky shifted solves, same m and M).  Bound: the
    shifted solves' residuals give a relative error <= tol sqrt(M / m) (twice that for the
    recurrence residual's drift), and float32 entries and products (M / m) eps32 (ten times
    that, as in the batched refresh tests)."""
    wl = I.batched()
    C = wl["chains"]
    inst = wl["instances"][::16]
    ns = [b["X"].shape[0] for b in inst]
    ds = [b["X"].shape[1] for b in inst]
    offs = [int(o) for o in np.cumsum([0] + ns[:-1])]
    xoffs = [int(o) for o in np.cumsum([0] + [a * b for a, b in zip(ns, ds)][:-1])]
    X = to_dev(np.concatenate([b["X"].ravel() for b in inst]), torch.float32)[:, None]
    xi = np.concatenate([b["xi"].ravel() for b in inst])
    th = np.concatenate([np.tile(b["theta"], C) for b in inst])
    tol = 1e-6
    r = gpk.phi_refresh_chains(X, to_dev(th, torch.float64), to_dev(xi, torch.float32), "ard", ns,
                               offs, C, d=ds, x_offsets=xoffs, tol=tol, maxit=3000,
                               mode=gpk.BATCHED)
    torch.cuda.synchronize()
    assert np.all(host(r["status"]) == 0)
    bi = int(np.argmin(ns))
    b, n = inst[bi], ns[bi]
    Xr = rounded(b["X"], torch.float32)
    bounds = host(r["bounds"]).reshape(-1, 2)[bi * C:(bi + 1) * C]
    m, M = bounds[0]
    assert np.all(bounds == bounds[0])
    assert m == pytest.approx(np.exp(b["theta"][-1]), rel=1e-15)
    M_ref = opoles.gershgorin_upper(Xr, b["theta"], "ard")
    assert M_ref <= M <= M_ref * (1 + 1e-4)  # widened past the float32 row sums' rounding
    ref = opoles.inv_sqrt_apply(Xr, b["theta"], "ard", rounded(b["xi"], torch.float32).T, M=M)
    phi = host(r["phi"])[C * offs[bi]:C * (offs[bi] + n)].reshape(C, n)
    bound = 2.0 * tol * np.sqrt(M / m) + 10 * (M / m) * 2.0 ** -24
    errs = [np.linalg.norm(phi[c] - ref[:, c]) / np.linalg.norm(ref[:, c]) for c in range(C)]
    print(f"batched refresh, N = {n}: max rel err {max(errs):.3e}, bound {bound:.3e}, "
          f"iterations {host(r['iters']).max()}")
    assert max(errs) < bound, (errs, bound)


def test_cheb2d_full_size_refresh_and_trajectories():
    """The cheb2d workload at full size (N = 3000 points in [-1, 1]^2, Chebyshev-amplitude SE with
    N_cheb = 4, FP64, 10 chains), launched as the benchmark's plain-CG run launches it: the 10
    chains' phi in one graph-mode gp_phi_refresh_chains launch, then their trajectories (3
    leapfrog steps of 0.03, update 0's pi and u) in one graph-mode gp_hmc_leapfrog launch.

    phi against the oracle's pole expansion with Cholesky shifted solves (same m and M), at the
    benchmark's tolerance and at a tight one.  Bound: each shifted system (A + lambda_p) x_p = xi
    stops at residual <= tol |xi| and A + lambda_p >= (m + lambda_p) I, so
    |delta phi| <= tol |xi| sum_p w_p / (m + lambda_p) ~ tol |xi| / sqrt(m), while
    |phi| >= |xi| / sqrt(M): relative error <= tol sqrt(M / m) (a factor 2 for the recurrence
    residual's drift).  Trajectories from the oracle's phi, CG at 1e-12, plain and with the
    benchmark's rank-500 Nystrom preconditioner, against the oracle's leapfrog with exact solves
    (one chain accepted, one rejected)."""
    wl = I.cheb2d()
    X, y, th0 = wl["X"], wl["y"], wl["theta"]
    n, C, nc = X.shape[0], wl["chains"], wl["n_cheb"]
    Xd = to_dev(X, torch.float64).reshape(-1, 1)
    xi = wl["xi"][0]  # (C, n): chain c's xi at c * n
    M_ref = opoles.gershgorin_upper(X, th0, "cheb")
    ref = opoles.inv_sqrt_apply(X, th0, "cheb", xi.T, M=M_ref * (1 + 1e-12))
    for tol in (1e-6, 1e-11):
        r = gpk.phi_refresh_chains(Xd, to_dev(np.tile(th0, C), torch.float64),
                                   to_dev(xi.ravel(), torch.float64), "cheb", [n], [0], C, d=[2],
                                   tol=tol, maxit=5000, n_cheb=nc, mode=gpk.GRAPH)
        torch.cuda.synchronize()
        assert np.all(host(r["status"]) == 0), tol
        bounds = host(r["bounds"]).reshape(-1, 2)
        m, M = bounds[0]
        assert np.all(bounds == bounds[0])
        assert M == pytest.approx(M_ref * (1 + 1e-12), rel=1e-12)
        phi = host(r["phi"]).reshape(C, n)
        bound = 2.0 * tol * np.sqrt(M / m) + 1e-13
        errs = [np.linalg.norm(phi[c] - ref[:, c]) / np.linalg.norm(ref[:, c]) for c in range(C)]
        print(f"cheb2d refresh tol {tol:g}: max rel err {max(errs):.3e}, bound {bound:.3e}, "
              f"iterations {host(r['iters']).max()}")
        assert max(errs) < bound, (tol, errs, bound)

    dt, ns = wl["dt"], wl["n_steps"]
    pi0, u = wl["pi"][0], wl["u"][0]
    nt = len(th0)
    # the benchmark's rank-500 factor at theta_0 (it changes iteration counts, not results)
    omega = to_dev(I.rng(I.WORKLOAD_SEEDS["cheb2d"], I.P_V).standard_normal((n, 500)), torch.float64)
    U, lam = gpk.nystrom(to_dev(X, torch.float64), to_dev(th0, torch.float64), omega, "cheb",
                         n_cheb=nc)
    oracle = {}
    for c in (0, C - 1):
        th1, pi1 = ohmc.leapfrog(X, "cheb", y, ref[:, c], th0, pi0[c], dt, ns)
        H0 = ohmc.hamiltonian(X, th0, "cheb", y, ref[:, c], pi0[c])
        H1 = ohmc.hamiltonian(X, th1, "cheb", y, ref[:, c], pi1)
        oracle[c] = (th1, pi1, H0, H1, ohmc.accept(H0, H1, u[c]))
    assert {o[4] for o in oracle.values()} == {True, False}
    iters = {}
    for precond in (None, (U, lam)):
        thd = to_dev(np.tile(th0, C), torch.float64)
        pid = to_dev(pi0.ravel(), torch.float64)
        x = torch.zeros(n * C, dtype=torch.float64, device=DEV)
        res = gpk.hmc_leapfrog(Xd, to_dev(y, torch.float64), to_dev(ref.T.ravel(), torch.float64),
                               thd, pid, x, "cheb", [n], [0], C, d=[2], u=to_dev(u, torch.float64),
                               n_steps=ns, dt=dt, cg_tol=1e-12, cg_maxit=5000, mode=gpk.GRAPH,
                               n_cheb=nc, precond=precond)
        torch.cuda.synchronize()
        th_out, pi_out = host(thd).reshape(C, nt), host(pid).reshape(C, nt)
        iters[precond is None] = host(res["cg_iters"])
        for c, (th1, pi1, H0, H1, acc) in oracle.items():
            assert int(res["status"][c]) == 0
            assert float(res["H0"][c]) == pytest.approx(H0, rel=1e-10)
            assert float(res["H1"][c]) == pytest.approx(H1, rel=1e-9)
            assert bool(res["accepted"][c]) == acc
            dth = np.max(np.abs(th_out[c] - (th1 if acc else th0)))
            dpi = np.max(np.abs(pi_out[c] - (pi1 if acc else pi0[c])))
            print(f"cheb2d chain {c}, preconditioned {precond is not None}: accepted {acc}, "
                  f"|theta - oracle| {dth:.3e}, |pi - oracle| {dpi:.3e}")
            assert dth < 1e-8 and dpi < 1e-8
    assert np.all(iters[False] < iters[True])
