"""gp_kmatvec_noalloc (the product of gp_kmatvec with its workspace in a device array the library
holds, for callers that cannot allocate) against gp_kmatvec, through the C ABI.

Two calls in a row on one stream, the second with a smaller input, each checked against the
workspace entry point on the same inputs at the FP32 tolerance (1e-5 relative per column, the
column-split count may differ and with it the order of the float sums), then an FP64 call at
1e-11; the first call is also checked against the oracle.  The first call's column tiles are
still in the array when the second runs, so a stale-contents dependence would show.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import gp as ogp
from paper_2412_20884_amd import gpk, inputs
from gpu_util import DEV, col_rel_err, host, rounded, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(kind, X, theta, V, col_shift=None):
    n, d = X.shape
    r = V.shape[1]
    k = gpk.make_kernel(kind, X)
    out = torch.full((n, r), float("nan"), dtype=X.dtype, device=DEV)
    st = gpk.lib().gp_kmatvec_noalloc(ctypes.byref(k), n, gpk._p(X), gpk._p(theta), r, gpk._p(V),
                                      V.stride(0), gpk._p(col_shift), gpk._p(out), out.stride(0),
                                      gpk._stream(X.device))
    gpk._check(st)
    return out


def _case(kind, n, d, r, seed, dtype, shift=False):
    if kind == "iso":
        p = inputs.iso_problem(n, d, seed, ell=0.15, sigma2=1e-2, r=r)
    else:
        p = inputs.ard_problem(n, d, seed, sigma2=1e-2, r=r)
    X = to_dev(rounded(p["X"], dtype), dtype)
    V = to_dev(rounded(p["V"], dtype), dtype)
    th = to_dev(p["theta"], torch.float64)
    cs = to_dev(np.linspace(0.0, 0.3, r), torch.float64) if shift else None
    return p, X, V, th, cs


def test_noalloc_matches_workspace_entry_point_two_calls():
    # call 1: n = 9000, R = 16 (matrix-core pass, several column tiles and a ragged tail)
    p1, X1, V1, th1, _ = _case("iso", 9000, 3, 16, 71, torch.float32)
    a1 = _noalloc("iso", X1, th1, V1)
    # call 2, smaller: n = 1700, ARD, R = 3 (VALU pass) with a per-column diagonal shift
    p2, X2, V2, th2, cs2 = _case("ard", 1700, 5, 3, 72, torch.float32, shift=True)
    a2 = _noalloc("ard", X2, th2, V2, cs2)
    b1 = gpk.kmatvec(X1, th1, V1, "iso")
    b2 = gpk.kmatvec(X2, th2, V2, "ard", col_shift=cs2)
    torch.cuda.synchronize()
    assert np.isfinite(host(a1)).all() and np.isfinite(host(a2)).all()
    e1 = col_rel_err(host(a1), host(b1))
    e2 = col_rel_err(host(a2), host(b2))
    print(f"noalloc vs gp_kmatvec: call 1 {e1:.2e}, call 2 {e2:.2e}")
    assert e1 < 1e-5 and e2 < 1e-5
    # call 1 against the oracle on the device-rounded inputs
    ref = ogp.matvec(rounded(p1["X"], torch.float32), p1["theta"], "iso",
                     rounded(p1["V"], torch.float32))
    assert col_rel_err(host(a1), ref) < 1e-5


def test_noalloc_fp64_and_repeat_is_bitwise():
    p, X, V, th, cs = _case("iso", 2500, 2, 8, 73, torch.float64, shift=True)
    a = _noalloc("iso", X, th, V, cs)
    b = gpk.kmatvec(X, th, V, "iso", col_shift=cs)
    a2 = _noalloc("iso", X, th, V, cs)
    torch.cuda.synchronize()
    assert col_rel_err(host(a), host(b)) < 1e-11
    assert torch.equal(a, a2)


def test_noalloc_rejects_what_does_not_fit():
    X = torch.zeros((400000, 3), dtype=torch.float32, device=DEV)
    V = torch.zeros((400000, 16), dtype=torch.float32, device=DEV)
    th = torch.zeros(3, dtype=torch.float64, device=DEV)
    with pytest.raises(gpk.GpkError) as ei:
        _noalloc("iso", X, th, V)
    assert ei.value.status == 4
