"""The hand-written backward passes of KMatVec and QuadForm against finite differences and the
FP64 oracle, including the ARD workload of N = 65,536 points in d = 8 with 16 right-hand sides."""
import numpy as np
import pytest
import torch

from oracle import gp as ogp
from paper_2412_20884_amd import autograd as ag, gpk, inputs as I
from tests.gpu_util import DEV, col_rel_err, grad_rel_err, host, rounded, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,d", [("iso", 2), ("ard", 3)])
def test_gradcheck_fp64(kind, d):
    p = I.iso_problem(40, d, 3, ell=0.4, r=3) if kind == "iso" else I.ard_problem(40, d, 3, r=3)
    X = to_dev(p["X"], torch.float64)
    th = to_dev(p["theta"], torch.float64).requires_grad_()
    V = to_dev(p["V"], torch.float64).requires_grad_()
    U = to_dev(p["U"], torch.float64).requires_grad_()
    assert torch.autograd.gradcheck(lambda t, v: ag.kmatvec(X, t, v, kind), (th, V), eps=1e-6, atol=1e-7)
    assert torch.autograd.gradcheck(lambda t, u, v: ag.quadform(X, t, u, v, kind), (th, U, V), eps=1e-6, atol=1e-7)


def test_backward_matches_oracle_fp32():
    p = I.ard_problem(3000, 5, 11, r=16)
    X = rounded(p["X"], torch.float32)
    V = rounded(p["V"], torch.float32)
    G = rounded(p["U"], torch.float32)
    th = p["theta"]
    thd = to_dev(th, torch.float64).requires_grad_()
    Vd = to_dev(V, torch.float32).requires_grad_()
    out = ag.kmatvec(to_dev(X, torch.float32), thd, Vd, "ard")
    out.backward(to_dev(G, torch.float32))
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, "ard", G, V)
    scale = ogp.quadform_grad(X, th, "ard", np.abs(G), np.abs(V))["grad"]
    assert col_rel_err(host(out.detach()), ref["AV"]) < 1e-5
    assert grad_rel_err(host(thd.grad), ref["grad"], scale) < 1e-5
    assert col_rel_err(host(Vd.grad), ref["AU"]) < 1e-5


def test_ard8_full_size_forward_backward():
    """N = 65,536, d = 8 ARD, 16 right-hand sides: forward and backward at full size.

    Sampled rows of A V and A G against the oracle; the theta-gradient restricted to a row
    sample (G zeroed outside it) against the oracle's row-restricted gradient, element by element.
    """
    w = I.ard8()
    X = rounded(w["X"], torch.float32)
    V = rounded(w["V"], torch.float32)
    G = rounded(w["G"], torch.float32)
    th = w["theta"]
    Xd = to_dev(X, torch.float32)
    thd = to_dev(th, torch.float64).requires_grad_()
    Vd = to_dev(V, torch.float32).requires_grad_()
    out = ag.kmatvec(Xd, thd, Vd, "ard")
    out.backward(to_dev(G, torch.float32))
    torch.cuda.synchronize()
    rows = np.random.default_rng(1).choice(X.shape[0], 48, replace=False)
    ref_av = ogp.matvec(X, th, "ard", V, rows=rows)
    ref_ag = ogp.matvec(X, th, "ard", G, rows=rows)
    rel = lambda a, b: np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0))
    assert rel(host(out.detach())[rows], ref_av) < 1e-5
    assert rel(host(Vd.grad)[rows], ref_ag) < 1e-5
    # row-restricted gradient: only rows in `rows` carry G, so sum_c G_c^T dA V_c runs over them
    Gm = np.zeros_like(G)
    Gm[rows] = G[rows]
    thd2 = to_dev(th, torch.float64).requires_grad_()
    out2 = ag.kmatvec(Xd, thd2, to_dev(V, torch.float32), "ard")
    out2.backward(to_dev(Gm, torch.float32))
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, "ard", Gm, V, rows=rows)["grad"]
    scale = ogp.quadform_grad(X, th, "ard", np.abs(Gm), np.abs(V), rows=rows)["grad"]
    assert grad_rel_err(host(thd2.grad), ref, scale) < 1e-5
