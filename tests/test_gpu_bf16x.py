"""GP_BF16X products: the coordinate cross term on the matrix cores in bfloat16 hi/lo.

Tolerance 3e-3 relative (the bfloat16 cross-term budget), on the whole product and on its
off-diagonal part (K - alpha I) V against that part's own norm: at d = 64 most kernel values
vanish and A is close to (alpha + sigma^2) I, so the check on the full product alone would be met
trivially.  d = 64 runs with the workload's length-scales and with long ones (8 .. 16) whose
off-diagonal part is substantial.
"""
import numpy as np
import pytest
import torch

from oracle import gp as ogp
from paper_2412_20884_amd import gpk, inputs as I
from tests.gpu_util import col_rel_err, grad_rel_err, host, rounded, to_dev

pytestmark = pytest.mark.gpu
TOL = 3e-3


def _offdiag(out, V, th):
    return out - (np.exp(th[0]) + np.exp(th[-1])) * V


EPS32 = 2.0 ** -24


def _offdiag_err(out, ref, V, th):
    """Column error of the off-diagonal part (K - alpha I) V relative to that part's own norm,
    returned as a ratio to the budget (pass: <= 1).  The diagonal pairs are added exactly; off the
    diagonal every kernel entry carries the norm expansion's error (a few eps32 |x~|^2 absolute in
    the exponent) and the float16 rounding of the scaled kernel value (2^-11 relative), far below
    3e-3 of the part itself.  The part is extracted from the float32 output as out - (alpha +
    sigma^2) V, so the output's own rounding (at most 2^-24 |out_i| per entry) is added to the
    budget: |err_c| <= 3e-3 |off_c| + 2 eps32 |out_c|, which matters only where the part is below
    ~1e-5 of the column (d = 64 at a few thousand points)."""
    num = np.linalg.norm(_offdiag(out, V, th) - _offdiag(ref, V, th), axis=0)
    den = TOL * np.linalg.norm(_offdiag(ref, V, th), axis=0) + 2 * EPS32 * np.linalg.norm(out, axis=0)
    return float(np.max(num / den))


# d = 64 twice: the workload's length-scales (0.5 .. 8: the off-diagonal part is ~1e-5 of a
# column at this N) and long ones (8 .. 16: scaled distances O(1), a substantial off-diagonal part)
@pytest.mark.parametrize("kind,d,lo,hi", [("iso", 3, None, None), ("ard", 8, 0.3, 3.0),
                                          ("ard", 33, 0.5, 8.0), ("ard", 64, 0.5, 8.0),
                                          ("ard", 64, 8.0, 16.0)])
@pytest.mark.parametrize("r", [1, 2, 16, 32])
def test_kmatvec_bf16x(kind, d, lo, hi, r):
    n = 3100
    if kind == "iso":
        p = I.iso_problem(n, d, 71, ell=0.15, r=r)
    else:
        p = I.ard_problem(n, d, 71 + d, lo=lo, hi=hi, r=r)
    X, V = rounded(p["X"], torch.float32), rounded(p["V"], torch.float32)
    th = p["theta"]
    out = gpk.kmatvec(to_dev(X, torch.float32), to_dev(th, torch.float64), to_dev(V, torch.float32),
                      kind, prec="bf16x")
    torch.cuda.synchronize()
    ref = ogp.matvec(X, th, kind, V)
    o = host(out)
    assert col_rel_err(o, ref) < TOL
    assert _offdiag_err(o, ref, V, th) <= 1.0


@pytest.mark.parametrize("kind,d,lo,hi", [("iso", 3, None, None), ("ard", 8, 0.5, 3.0),
                                          ("ard", 64, 0.5, 8.0), ("ard", 64, 8.0, 16.0)])
@pytest.mark.parametrize("r", [2, 16])
def test_quadform_bf16x(kind, d, lo, hi, r):
    n = 2600
    if kind == "iso":
        p = I.iso_problem(n, d, 81, ell=0.15, r=r)
    else:
        p = I.ard_problem(n, d, 81 + d, lo=lo, hi=hi, r=r)
    X, U = rounded(p["X"], torch.float32), rounded(p["U"], torch.float32)
    th = p["theta"]
    w = np.linspace(-0.5, 0.5, r) + (0.25 if r > 1 else 1.0)
    Ud = to_dev(U, torch.float32)
    res = gpk.quadform_grad(to_dev(X, torch.float32), to_dev(th, torch.float64), Ud, Ud,
                            to_dev(w, torch.float64), kind, prec="bf16x", want_AU=True)
    torch.cuda.synchronize()
    ref = ogp.quadform_grad(X, th, kind, U, U, w)
    scale = ogp.quadform_grad(X, th, kind, np.abs(U), np.abs(U), np.abs(w))["grad"]
    au = host(res["AU"])
    assert col_rel_err(au, ref["AU"]) < TOL
    assert _offdiag_err(au, ref["AU"], U, th) <= 1.0
    # the alpha component carries the diagonal's alpha sum_c w_c |u_c|^2 (exact on the device):
    # compare it relative to its off-diagonal scale alone
    K0 = np.exp(th[0])
    offs = scale.copy()
    offs[0] = scale[0] - K0 * np.sum(np.abs(w) * np.sum(U * U, axis=0))
    assert grad_rel_err(host(res["grad"]), ref["grad"], offs) < TOL
