"""Parity at the full sizes of the workloads, in the launch configuration the benchmark times.

The oracle computes sampled rows one by one (all N columns each); sums over all N^2 pairs are
checked through identities that hold at any size, and the theta-gradient element by element on
a row sample (the left operand zeroed outside it, so the gradient is the oracle's
row-restricted one).  The batched trajectories are checked for exact agreement between the
graph replay and the persistent launch, and against the plain single-chain form.
"""
import numpy as np
import pytest
import torch

from oracle import gp as ogp
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
