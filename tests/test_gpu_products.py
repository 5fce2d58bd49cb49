"""GPU parity of gp_kmatvec and gp_quadform_grad against the FP64 oracle.

Inputs are seeded and synthetic; the oracle sees the values the device holds (inputs rounded to
the device precision and converted exactly to float64), so the measured error is the kernels'
arithmetic error.  Tolerances: FP64 1e-11 relative; FP32 1e-5 relative, per column in the 2-norm
and per entry against (|A| |V|)_ic (one wrong row cannot hide in a column norm); gradients
relative to the condition-aware scale sum_c |w_c| |u_c|^T |dA/dtheta| |v_c|.
Sizes span several 256-row blocks, ragged tails and the column-split path.
"""
import numpy as np
import pytest
import torch

from oracle import gp as ogp
from paper_2412_20884_amd import gpk, inputs as I
from tests.gpu_util import DEV, col_rel_err, comp_rel_err, grad_rel_err, host, rounded, to_dev

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-11, torch.float32: 1e-5}


def _problem(kind, n, d, seed, r, dist=None):
    if kind == "iso":
        return I.iso_problem(n, d, seed, ell=0.3, sigma2=1e-2, r=r)
    return I.ard_problem(n, d, seed, r=r)


def _grad_scale(X, th, kind, U, V, w):
    return ogp.quadform_grad(X, th, kind, np.abs(U), np.abs(V), np.abs(w))["grad"]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_kmatvec_small_fp64_workload(dtype):
    w = I.small_fp64()
    X, V = rounded(w["X"], dtype), rounded(w["V"], dtype)
    out = gpk.kmatvec(to_dev(X, dtype), to_dev(w["theta"], torch.float64), to_dev(V, dtype), "iso")
    torch.cuda.synchronize()
    ref = ogp.matvec(X, w["theta"], "iso", V)
    assert col_rel_err(host(out), ref) < TOL[dtype]
    assert comp_rel_err(host(out), ref, ogp.matvec(X, w["theta"], "iso", np.abs(V))) < TOL[dtype]


@pytest.mark.parametrize("n", [1, 7, 300, 1000, 4099, 9001])
@pytest.mark.parametrize("r", [1, 3, 8, 32])
def test_kmatvec_iso_f32_sizes(n, r):
    p = _problem("iso", n, 3, 100 + n, r)
    X, V = rounded(p["X"], torch.float32), rounded(p["V"], torch.float32)
    out = gpk.kmatvec(to_dev(X, torch.float32), to_dev(p["theta"], torch.float64),
                      to_dev(V, torch.float32), "iso")
    torch.cuda.synchronize()
    ref = ogp.matvec(X, p["theta"], "iso", V)
    assert col_rel_err(host(out), ref) < TOL[torch.float32]
    assert comp_rel_err(host(out), ref, ogp.matvec(X, p["theta"], "iso", np.abs(V))) < TOL[torch.float32]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("d", [1, 5, 8, 16, 33])
def test_kmatvec_ard_dims_shift_no_noise(dtype, d):
    p = _problem("ard", 2500, d, 7 + d, 4)
    X, V = rounded(p["X"], dtype), rounded(p["V"], dtype)
    shift = np.array([0.0, 0.3, 1.5, 7.0])
    Xd, Vd, th = to_dev(X, dtype), to_dev(V, dtype), to_dev(p["theta"], torch.float64)
    out = gpk.kmatvec(Xd, th, Vd, "ard", col_shift=to_dev(shift, torch.float64))
    nn = gpk.kmatvec(Xd, th, Vd, "ard", no_noise=True)
    torch.cuda.synchronize()
    ref = ogp.matvec(X, p["theta"], "ard", V, col_shift=shift)
    ref_nn = ogp.matvec(X, p["theta"], "ard", V, no_noise=True)
    assert col_rel_err(host(out), ref) < TOL[dtype]
    assert col_rel_err(host(nn), ref_nn) < TOL[dtype]
    absref = ogp.matvec(X, p["theta"], "ard", np.abs(V), col_shift=shift)
    assert comp_rel_err(host(out), ref, absref) < TOL[dtype]
    assert comp_rel_err(host(nn), ref_nn, ogp.matvec(X, p["theta"], "ard", np.abs(V), no_noise=True)) < TOL[dtype]


def test_kmatvec_wide_r_and_strided_operands():
    # r > 32 runs in several column chunks; V and out are column slices of wider buffers
    p = _problem("iso", 1500, 2, 5, 45)
    X, V = rounded(p["X"], torch.float32), rounded(p["V"], torch.float32)
    big = torch.zeros((1500, 50), dtype=torch.float32, device=DEV)
    big[:, 2:47] = to_dev(V, torch.float32)
    outbig = torch.full((1500, 60), 7.0, dtype=torch.float32, device=DEV)
    gpk.kmatvec(to_dev(X, torch.float32), to_dev(p["theta"], torch.float64), big[:, 2:47], "iso",
                out=outbig[:, 5:50])
    torch.cuda.synchronize()
    ref = ogp.matvec(X, p["theta"], "iso", V)
    assert col_rel_err(host(outbig[:, 5:50]), ref) < 1e-5
    assert torch.all(outbig[:, :5] == 7.0) and torch.all(outbig[:, 50:] == 7.0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind,d", [("iso", 2), ("iso", 3), ("ard", 4), ("ard", 8)])
@pytest.mark.parametrize("n", [777, 5000])
def test_quadform_symmetric(dtype, kind, d, n):
    p = _problem(kind, n, d, 31 + d + n, 5)
    X, U = rounded(p["X"], dtype), rounded(p["U"], dtype)
    w = np.array([0.5, -1.0, 2.0, 0.25, -0.75])
    th = p["theta"]
    Ud = to_dev(U, dtype)
    res = gpk.quadform_grad(to_dev(X, dtype), to_dev(th, torch.float64), Ud, Ud,
                            to_dev(w, torch.float64), kind, want_AU=True, want_AV=True)
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, kind, U, U, w)
    scale = _grad_scale(X, th, kind, U, U, w)
    tol = TOL[dtype]
    assert grad_rel_err(host(res["grad"]), ref["grad"], scale) < tol
    qscale = np.diag(np.abs(U).T @ ogp.matvec(X, th, kind, np.abs(U)))
    assert np.max(np.abs(host(res["quad"]) - ref["quad"]) / qscale) < tol
    assert col_rel_err(host(res["AU"]), ref["AU"]) < tol
    assert col_rel_err(host(res["AV"]), ref["AV"]) < tol
    assert comp_rel_err(host(res["AU"]), ref["AU"], ogp.matvec(X, th, kind, np.abs(U))) < tol


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("want", ["AU", "AV", "both", "none"])
def test_quadform_unsymmetric(dtype, want):
    p = _problem("ard", 3001, 3, 77, 3)
    X, U, V = (rounded(p[k], dtype) for k in ("X", "U", "V"))
    th = p["theta"]
    res = gpk.quadform_grad(to_dev(X, dtype), to_dev(th, torch.float64), to_dev(U, dtype),
                            to_dev(V, dtype), None, "ard", want_AU=want in ("AU", "both"),
                            want_AV=want in ("AV", "both"))
    torch.cuda.synchronize()
    w = np.ones(3)
    ref = ogp.quadform_grad(X, th, "ard", U, V, w)
    tol = TOL[dtype]
    assert grad_rel_err(host(res["grad"]), ref["grad"], _grad_scale(X, th, "ard", U, V, w)) < tol
    qscale = np.abs(U).T @ ogp.matvec(X, th, "ard", np.abs(V))
    assert np.max(np.abs(host(res["quad"]) - ref["quad"]) / np.diag(qscale)) < tol
    if want in ("AU", "both"):
        assert col_rel_err(host(res["AU"]), ref["AU"]) < tol
    if want in ("AV", "both"):
        assert col_rel_err(host(res["AV"]), ref["AV"]) < tol


def test_quadform_empty_and_single_point():
    th = to_dev(np.log([1.5, 0.3, 0.1]), torch.float64)
    X0 = torch.zeros((0, 2), dtype=torch.float64, device=DEV)
    U0 = torch.zeros((0, 2), dtype=torch.float64, device=DEV)
    res = gpk.quadform_grad(X0, th, U0, U0, None, "iso")
    torch.cuda.synchronize()
    assert torch.all(res["grad"] == 0) and torch.all(res["quad"] == 0)
    X1 = to_dev([[0.2, 0.4]], torch.float64)
    U1 = to_dev([[2.0, -1.0]], torch.float64)
    res = gpk.quadform_grad(X1, th, U1, U1, None, "iso", want_AU=True)
    torch.cuda.synchronize()
    # A = [alpha + s2]; q_c = (alpha + s2) u_c^2; grad = (alpha sum u^2, 0, s2 sum u^2)
    np.testing.assert_allclose(host(res["quad"]), [1.6 * 4.0, 1.6 * 1.0], rtol=1e-14)
    np.testing.assert_allclose(host(res["grad"]), [1.5 * 5.0, 0.0, 0.1 * 5.0], rtol=1e-14, atol=1e-300)


def test_determinism_bitwise():
    p = _problem("iso", 6000, 3, 3, 8)
    X = to_dev(p["X"], torch.float32)
    U = to_dev(p["U"], torch.float32)
    th = to_dev(p["theta"], torch.float64)
    a = gpk.quadform_grad(X, th, U, U, None, "iso", want_AU=True)
    b = gpk.quadform_grad(X, th, U, U, None, "iso", want_AU=True)
    torch.cuda.synchronize()
    assert torch.equal(a["grad"], b["grad"]) and torch.equal(a["AU"], b["AU"])
    assert torch.equal(a["quad"], b["quad"])


# ---- matrix-core (fp16 hi/lo split) path: float inputs, 8 <= R <= 32, d <= 16 ---------------

@pytest.mark.parametrize("kind,d", [("iso", 1), ("iso", 3), ("iso", 4), ("ard", 2), ("ard", 8),
                                    ("ard", 13), ("ard", 16)])
@pytest.mark.parametrize("r", [8, 16, 20, 32])
@pytest.mark.parametrize("n", [300, 5003])
def test_quadform_mfma_symmetric(kind, d, r, n):
    p = _problem(kind, n, d, 500 + 7 * d + r + n, r)
    X, U = rounded(p["X"], torch.float32), rounded(p["U"], torch.float32)
    w = np.linspace(-1.0, 2.0, r)
    th = p["theta"]
    Ud = to_dev(U, torch.float32)
    res = gpk.quadform_grad(to_dev(X, torch.float32), to_dev(th, torch.float64), Ud, Ud,
                            to_dev(w, torch.float64), kind, want_AU=True)
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, kind, U, U, w)
    assert col_rel_err(host(res["AU"]), ref["AU"]) < 1e-5
    assert grad_rel_err(host(res["grad"]), ref["grad"], _grad_scale(X, th, kind, U, U, w)) < 1e-5
    qscale = np.diag(np.abs(U).T @ ogp.matvec(X, th, kind, np.abs(U)))
    assert np.max(np.abs(host(res["quad"]) - ref["quad"]) / qscale) < 1e-5


@pytest.mark.parametrize("want", ["AU", "AV", "both"])
@pytest.mark.parametrize("n", [1000, 6000])
def test_quadform_mfma_unsymmetric(want, n):
    p = _problem("ard", n, 6, 91 + n, 16)
    X, U, V = (rounded(p[k], torch.float32) for k in ("X", "U", "V"))
    th = p["theta"]
    w = np.linspace(0.5, 1.5, 16)
    res = gpk.quadform_grad(to_dev(X, torch.float32), to_dev(th, torch.float64),
                            to_dev(U, torch.float32), to_dev(V, torch.float32),
                            to_dev(w, torch.float64), "ard", want_AU=want in ("AU", "both"),
                            want_AV=want in ("AV", "both"))
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, "ard", U, V, w)
    assert grad_rel_err(host(res["grad"]), ref["grad"], _grad_scale(X, th, "ard", U, V, w)) < 1e-5
    qscale = np.abs(U).T @ ogp.matvec(X, th, "ard", np.abs(V))
    assert np.max(np.abs(host(res["quad"]) - ref["quad"]) / np.diag(qscale)) < 1e-5
    if want in ("AU", "both"):
        assert col_rel_err(host(res["AU"]), ref["AU"]) < 1e-5
    if want in ("AV", "both"):
        assert col_rel_err(host(res["AV"]), ref["AV"]) < 1e-5


@pytest.mark.parametrize("mag", [1e-6, 1e5])
@pytest.mark.parametrize("log_alpha", [-4.0, 6.0])
def test_mfma_operand_scaling(mag, log_alpha):
    # operands far from unit scale and alpha far from 1 exercise the power-of-two scaling
    p = I.iso_problem(2100, 2, 17, ell=0.2, sigma2=1e-2, r=16)
    th = p["theta"].copy()
    th[0] = log_alpha
    X = rounded(p["X"], torch.float32)
    V = rounded(p["V"] * mag, torch.float32)
    out = gpk.kmatvec(to_dev(X, torch.float32), to_dev(th, torch.float64), to_dev(V, torch.float32), "iso")
    res = gpk.quadform_grad(to_dev(X, torch.float32), to_dev(th, torch.float64),
                            to_dev(V, torch.float32), None, None, "iso")
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, "iso", V, V)
    assert col_rel_err(host(out), ref["AV"]) < 1e-5
    scale = _grad_scale(X, th, "iso", V, V, np.ones(16))
    assert grad_rel_err(host(res["grad"]), ref["grad"], scale) < 1e-5


@pytest.mark.parametrize("kind,d,r", [("iso", 3, 32), ("ard", 8, 16), ("iso", 2, 1)])
def test_autotuned_config_keeps_parity(kind, d, r):
    """After tuning a problem class the products still match the oracle."""
    n = 4500
    gpk.tune_clear()
    gpk.tune(kind, d, n, r, torch.float32, with_grad=True)
    gpk.tune(kind, d, n, r, torch.float32, with_grad=False)
    assert gpk.tune_entries() == 2
    p = _problem(kind, n, d, 61 + d, r)
    X, U = rounded(p["X"], torch.float32), rounded(p["U"], torch.float32)
    th = p["theta"]
    Ud = to_dev(U, torch.float32)
    res = gpk.quadform_grad(to_dev(X, torch.float32), to_dev(th, torch.float64), Ud, Ud, None, kind,
                            want_AU=True)
    out = gpk.kmatvec(to_dev(X, torch.float32), to_dev(th, torch.float64), Ud, kind)
    torch.cuda.synchronize()
    gpk.tune_clear()
    ref = ogp.quadform_grad(X, th, kind, U, U)
    assert col_rel_err(host(res["AU"]), ref["AU"]) < 1e-5
    assert col_rel_err(host(out), ref["AU"]) < 1e-5
    assert grad_rel_err(host(res["grad"]), ref["grad"], _grad_scale(X, th, kind, U, U, np.ones(r))) < 1e-5


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind,d,r", [("iso", 2, 16), ("ard", 5, 7), ("ard", 3, 17)])
def test_quadform_unsymmetric_both_products(dtype, kind, d, r):
    """U != V with A U and A V: one pass of 2r columns for r <= 16 (the matrix-core path at
    2r >= 8 in float), two passes for r = 17; weights of both signs."""
    p = _problem(kind, 2300, d, 97 + r, r)
    X, U, V = (rounded(p[k], dtype) for k in ("X", "U", "V"))
    th = p["theta"]
    w = np.linspace(-1.0, 1.5, r)
    res = gpk.quadform_grad(to_dev(X, dtype), to_dev(th, torch.float64), to_dev(U, dtype),
                            to_dev(V, dtype), to_dev(w, torch.float64), kind, want_AU=True,
                            want_AV=True)
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, kind, U, V, w)
    tol = TOL[dtype]
    assert grad_rel_err(host(res["grad"]), ref["grad"], _grad_scale(X, th, kind, U, V, w)) < tol
    qscale = np.diag(np.abs(U).T @ ogp.matvec(X, th, kind, np.abs(V)))
    assert np.max(np.abs(host(res["quad"]) - ref["quad"]) / qscale) < tol
    assert comp_rel_err(host(res["AU"]), ref["AU"], ogp.matvec(X, th, kind, np.abs(U))) < tol
    assert comp_rel_err(host(res["AV"]), ref["AV"], ogp.matvec(X, th, kind, np.abs(V))) < tol
