"""The C-ABI library loads, exports every symbol include/gpk.h declares, and rejects bad
arguments on the host before touching a GPU (so these run on a CPU-only machine)."""
import ctypes
import os
import re

import pytest

from paper_2412_20884_amd import gpk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpk.h")

pytestmark = pytest.mark.skipif(not os.path.exists(gpk.LIB_PATH), reason="libgpk.so not built")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    syms = declared_symbols()
    assert set(syms) == set(gpk.EXPORTED), syms
    L = ctypes.CDLL(gpk.LIB_PATH)
    for s in syms:
        assert hasattr(L, s), s


def test_status_strings_and_n_theta():
    L = gpk.lib()
    assert L.gp_status_string(0) == b"GP_OK"
    assert L.gp_status_string(4) == b"GP_ERR_WORKSPACE"
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 3, 0))) == 3
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.ARD, gpk.F32, 8, 0))) == 10
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(7, gpk.F32, 8, 0))) == -1
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.ARD, gpk.F32, 65, 0))) == -1
    # Chebyshev-amplitude kernel: N_cheb^d + 2 hyperparameters, at most 64 terms
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.CHEB, gpk.F32, 1, 0, 2))) == 4
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.CHEB, gpk.F64, 3, 0, 4))) == 66
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.CHEB, gpk.F32, 2, 0, 9))) == -1
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.CHEB, gpk.F32, 2, 0, 0))) == -1
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.CHEB, gpk.F32, 64, 0, 1))) == 3
    assert L.gp_n_theta(ctypes.byref(gpk.Kernel(gpk.CHEB, gpk.F32, 7, 0, 2))) == -1


def _kmv(k, n=10, X=1, th=1, r=2, V=4096, ldv=2, out=1 << 20, ldo=2, ws=8, wsb=1 << 30):
    L = gpk.lib()
    vp = ctypes.c_void_p
    return L.gp_kmatvec(k, n, vp(X), vp(th), r, vp(V), ldv, None, vp(out), ldo, vp(ws), wsb, None)


def test_kmatvec_validation():
    L = gpk.lib()
    good = ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 3, 0))
    assert _kmv(None) == 1
    assert b"NULL" in L.gp_last_error()
    assert _kmv(ctypes.byref(gpk.Kernel(5, gpk.F32, 3, 0))) == 1
    assert _kmv(ctypes.byref(gpk.Kernel(gpk.ISO, 9, 3, 0))) == 1
    assert _kmv(ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 0, 0))) == 2
    assert _kmv(ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 3, 8))) == 1
    assert _kmv(good, n=-1) == 2
    assert _kmv(good, r=-1) == 2
    assert _kmv(good, X=0) == 1
    assert _kmv(good, ldv=1) == 2
    assert _kmv(good, ldo=1) == 2
    # out overlapping V
    assert _kmv(good, V=4096, out=4100) == 1
    # workspace missing / too small
    assert _kmv(good, ws=0) == 4
    assert _kmv(good, wsb=16) == 4
    assert b"workspace" in L.gp_last_error()
    # empty problems are a no-op and succeed without touching memory
    assert _kmv(good, n=0, X=0, V=0, out=0, ws=0) == 0
    assert _kmv(good, r=0, X=0, V=0, out=0, ws=0) == 0


def test_quadform_validation():
    L = gpk.lib()
    vp = ctypes.c_void_p
    k = ctypes.byref(gpk.Kernel(gpk.ARD, gpk.F32, 4, 0))

    def q(kk=k, n=10, r=2, U=4096, V=8192, grad=1, quad=0, AU=0, AV=0, ldau=2, wsb=1 << 30):
        return L.gp_quadform_grad(kk, n, vp(1), vp(1), r, vp(U), 2, vp(V), 2, None, vp(grad),
                                  vp(quad), vp(AU), ldau, vp(AV), 2, vp(16), wsb, None)

    assert q(r=0) == 2
    assert q(r=33) == 2
    assert q(grad=0) == 1
    # GP_NO_NOISE is accepted (the form in K alone): the call gets as far as the workspace check
    assert q(kk=ctypes.byref(gpk.Kernel(gpk.ARD, gpk.F32, 4, gpk.NO_NOISE)), wsb=8) == 4
    assert q(AU=4096 + 8) == 1          # AU overlaps U
    assert q(AU=1 << 20, ldau=1) == 2
    assert q(wsb=8) == 4


def test_workspace_size_monotone():
    L = gpk.lib()
    k = ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 3, 0))
    a = L.gp_workspace_size(k, 1000, 4)
    b = L.gp_workspace_size(k, 100000, 4)
    assert 0 < a < b
    assert L.gp_workspace_size(k, 0, 4) == 0
    assert L.gp_workspace_size(None, 10, 4) == 0


def test_tune_table_json_roundtrip(tmp_path):
    # the tuning table loads from and saves to JSON without a GPU
    gpk.tune_clear()
    src = tmp_path / "in.json"
    src.write_text('{"version": 1, "entries": [\n'
                   ' {"op": 1, "prec": 1, "kind": 0, "dp": 4, "rb": 32, "nb": 20, "splits": 2, "ib": 2, "ms": 780.5},\n'
                   ' {"op": 0, "prec": 0, "kind": 1, "dp": 8, "rb": 1, "nb": 12, "splits": 8, "ib": 1, "ms": 0.25},\n'
                   ' {"op": 0, "prec": 0, "kind": 1, "dp": 8, "rb": 1, "nb": 13, "splits": 0, "ib": 1, "ms": 0.25}\n'
                   ']}\n')
    gpk.tune_load(src)
    assert gpk.tune_entries() == 2          # the entry with splits = 0 is rejected
    out = tmp_path / "out.json"
    gpk.tune_save(out)
    gpk.tune_clear()
    assert gpk.tune_entries() == 0
    gpk.tune_load(out)
    assert gpk.tune_entries() == 2
    text = out.read_text()
    assert '"splits": 2' in text and '"nb": 12' in text
    gpk.tune_clear()
    L = gpk.lib()
    assert L.gp_tune_load(b"/nonexistent/x.json") == 1


def test_trajectory_tune_entries_and_validation(tmp_path):
    # trajectory entries (op 2) carry the launch configuration; a wave count outside 1..4 is
    # rejected on load
    gpk.tune_clear()
    src = tmp_path / "traj.json"
    src.write_text('{"version": 1, "entries": [\n'
                   ' {"op": 2, "prec": 1, "kind": 1, "dp": 16, "rb": 0, "nb": 14, "splits": 1, "ib": 1, '
                   '"ms": 12.5, "waves": 2, "cpt_lo": 4, "cpt_hi": 1},\n'
                   ' {"op": 2, "prec": 1, "kind": 1, "dp": 8, "rb": 0, "nb": 14, "splits": 1, "ib": 1, '
                   '"ms": 12.5, "waves": 9, "cpt_lo": 4, "cpt_hi": 1}\n'
                   ']}\n')
    gpk.tune_load(src)
    assert gpk.tune_entries() == 1
    out = tmp_path / "traj_out.json"
    gpk.tune_save(out)
    text = out.read_text()
    assert '"waves": 2' in text and '"cpt_lo": 4' in text and '"cpt_hi": 1' in text
    gpk.tune_clear()
    # validation happens before any HIP call
    L = gpk.lib()
    k = gpk.Kernel(gpk.ARD, gpk.F32, 4, 0, 0)
    prm = gpk.HmcParams(1, 0.0, 1e-6, 4, gpk.BATCHED, None, 0, None, None, None)
    npts = (ctypes.c_int64 * 2)(1000, 500)
    offs = (ctypes.c_int64 * 2)(0, 1000)
    dd = (ctypes.c_int32 * 2)(4, 16)
    b = gpk.Batch(2, 2, npts, offs, dd, None)
    nb = L.gp_tune_hmc_workspace_size(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b))
    assert nb > L.gp_hmc_workspace_size(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b))
    assert L.gp_tune_hmc(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b), None, 0, None) == 4
    bad = gpk.Batch(2, 0, npts, offs, dd, None)
    assert L.gp_tune_hmc_workspace_size(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(bad)) == 0
    assert L.gp_tune_hmc(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(bad), None, 0, None) == 2


def test_phi_chains_validation():
    """gp_phi_refresh_chains checks its parameters, the batch and the workspace before any HIP
    call; its workspace holds the trajectory workspace's vectors plus the shifted directions."""
    L = gpk.lib()
    vp = ctypes.c_void_p
    k = gpk.Kernel(gpk.ARD, gpk.F32, 4, 0, 0)
    npts = (ctypes.c_int64 * 2)(1000, 500)
    offs = (ctypes.c_int64 * 2)(0, 1000)
    dd = (ctypes.c_int32 * 2)(4, 16)
    b = gpk.Batch(2, 3, npts, offs, dd, None)
    hp = gpk.HmcParams(0, 0.0, 1e-6, 100, gpk.BATCHED, None, 0, None, None, None)

    def ws_size(pp, mode=gpk.BATCHED, kk=k, bb=b):
        return L.gp_phi_chains_workspace_size(ctypes.byref(kk), ctypes.byref(pp), mode, ctypes.byref(bb))

    def call(pp, kk=k, xi=1 << 12, phi=1 << 40, ws=None, wsb=0, mode=gpk.BATCHED):
        return L.gp_phi_refresh_chains(ctypes.byref(kk), ctypes.byref(pp), mode, ctypes.byref(b),
                                       vp(1 << 30), vp(1 << 31), vp(xi), vp(phi), vp(1 << 32), None,
                                       None, vp(ws) if ws else None, wsb, None)

    ok = gpk.PhiParams(15, 1e-6, 100, 0.0, 0, None, None)
    n15 = ws_size(ok)
    traj = L.gp_hmc_workspace_size(ctypes.byref(k), ctypes.byref(hp), ctypes.byref(b))
    # 6 chains of 1000 / 500 float rows, 15 directions each
    assert n15 >= traj + 4 * 15 * 3 * (1000 + 500)
    assert ws_size(gpk.PhiParams(30, 1e-6, 100, 0.0, 0, None, None)) > n15
    assert ws_size(ok, mode=gpk.PLAIN) > 0 and ws_size(ok, mode=7) == 0
    for bad in (gpk.PhiParams(0, 1e-6, 100, 0.0, 0, None, None),
                gpk.PhiParams(65, 1e-6, 100, 0.0, 0, None, None),
                gpk.PhiParams(15, 0.0, 100, 0.0, 0, None, None),
                gpk.PhiParams(15, 1e-6, 0, 0.0, 0, None, None),
                gpk.PhiParams(15, 1e-6, 100, float("nan"), 0, None, None)):
        assert ws_size(bad) == 0
        assert call(bad) == 1
    assert call(gpk.PhiParams(15, 1e-6, 100, 0.0, 5, vp(8), vp(8))) == 3
    assert call(ok, kk=gpk.Kernel(gpk.ARD, gpk.F32, 4, gpk.NO_NOISE, 0)) == 1
    assert call(ok, kk=gpk.Kernel(gpk.CHEB, gpk.BF16X, 2, 0, 2)) == 3
    assert call(ok) == 4                                   # no workspace
    assert call(ok, ws=1 << 20, wsb=n15 - 1) == 4          # one byte short
    assert call(ok, xi=1 << 12, phi=(1 << 12) + 8) == 1    # phi overlaps xi
    bad_b = gpk.Batch(2, 0, npts, offs, dd, None)
    assert ws_size(ok, bb=bad_b) == 0


def test_cheb_workspace_and_tuner():
    L = gpk.lib()
    k = ctypes.byref(gpk.Kernel(gpk.CHEB, gpk.F32, 2, 0, 3))
    se = ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 2, gpk.NO_NOISE, 0))
    # the Chebyshev path holds the SE workspace plus amplitudes and four scaled n x r blocks
    assert L.gp_workspace_size(k, 5000, 4) > L.gp_workspace_size(se, 5000, 4) + 4 * 5000 * 4 * 4
    assert L.gp_workspace_size(ctypes.byref(gpk.Kernel(gpk.CHEB, gpk.F32, 2, 0, 9)), 5000, 4) == 0
    assert L.gp_tune_workspace_size(k, 5000, 4) == 0
    assert L.gp_tune_products(k, 5000, 4, 1, None, 0, None) == 3


def test_nystrom_and_pcg_validation():
    L = gpk.lib()
    vp = ctypes.c_void_p
    k = ctypes.byref(gpk.Kernel(gpk.ARD, gpk.F32, 4, 0))
    nn = ctypes.byref(gpk.Kernel(gpk.ARD, gpk.F32, 4, gpk.NO_NOISE))

    def ny(kk=k, n=100, rank=5, om=4096, U=1 << 20, lam=8, ws=8, wsb=1 << 40):
        return L.gp_nystrom(kk, n, vp(1), vp(1), rank, vp(om), vp(U), vp(lam), vp(ws), wsb, None)

    assert ny(rank=0) == 2
    assert ny(rank=101) == 2
    assert ny(rank=513, n=10000) == 2
    assert ny(n=0) == 2
    assert ny(lam=0) == 1
    assert ny(U=4096 + 16) == 1        # U overlaps omega
    assert ny(ws=0) == 4
    assert L.gp_nystrom_workspace_size(k, 1000, 10) > 3 * 1000 * 10 * 4
    assert L.gp_nystrom_workspace_size(k, 1000, 0) == 0

    def pcg(kk=k, n=100, r=2, B=4096, ldb=2, x=1 << 20, ldx=2, rank=0, U=0, lam=0, tol=1e-6,
            maxit=10, ws=8, wsb=1 << 40):
        return L.gp_pcg_solve(kk, n, vp(1), vp(1), r, vp(B), ldb, vp(x), ldx, None, rank, vp(U),
                              vp(lam), tol, maxit, None, None, vp(ws), wsb, None)

    assert pcg(kk=nn) == 1
    assert pcg(r=0) == 2
    assert pcg(r=33) == 2
    assert pcg(rank=3) == 1              # rank > 0 without U, lam
    assert pcg(ldb=1) == 2
    assert pcg(tol=0.0) == 1
    assert pcg(x=4096 + 8) == 1          # x overlaps B
    assert pcg(ws=0) == 4
    assert L.gp_pcg_workspace_size(k, 1000, 4, 20) > L.gp_pcg_workspace_size(k, 1000, 4, 0)
    assert L.gp_pcg_workspace_size(nn, 1000, 4, 0) == 0


def test_implicit_validation():
    L = gpk.lib()
    vp = ctypes.c_void_p
    k = ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F64, 2, 0))

    def imp(kk=k, prm=None, n=100, rank=0, U=0, lam=0, ws=8, wsb=1 << 40, y=4096):
        prm = prm or gpk.ImplicitParams(3, 0.1, 10, 1e-8, 100, 1e-6, 100, 10)
        return L.gp_hmc_implicit(kk, ctypes.byref(prm), n, vp(1), vp(y), vp(8192), vp(16), vp(32),
                                 vp(1 << 20), None, rank, vp(U), vp(lam), vp(64), vp(72), vp(80),
                                 vp(84), None, vp(ws), wsb, None)

    assert imp(kk=None) == 1
    assert imp(kk=ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F64, 2, gpk.NO_NOISE))) == 1
    for bad in (gpk.ImplicitParams(-1, 0.1, 10, 1e-8, 100, 1e-6, 100, 10),
                gpk.ImplicitParams(3, 0.1, 21, 1e-8, 100, 1e-6, 100, 10),
                gpk.ImplicitParams(3, 0.1, 10, 0.0, 100, 1e-6, 100, 10),
                gpk.ImplicitParams(3, 0.1, 10, 1e-8, 0, 1e-6, 100, 10),
                gpk.ImplicitParams(3, 0.1, 10, 1e-8, 100, 1e-6, 100, 0)):
        assert imp(prm=bad) == 1
    assert imp(n=0) == 2
    assert imp(rank=5) == 1          # rank without U, lam
    assert imp(y=0) == 1
    assert imp(ws=0) == 4
    prm = gpk.ImplicitParams(3, 0.1, 10, 1e-8, 100, 1e-6, 100, 10)
    prm0 = gpk.ImplicitParams(3, 0.1, 0, 1e-8, 100, 1e-6, 100, 10)
    assert L.gp_implicit_workspace_size(k, ctypes.byref(prm), 1000, 0) > \
        L.gp_implicit_workspace_size(k, ctypes.byref(prm0), 1000, 0) + 2 * 9 * 1000 * 8 - 1024


# ---- binding-side validation (no kernel launches: CPU tensors never reach the library) ------

def _t(*shape, dtype=None):
    import torch
    return torch.zeros(*shape, dtype=dtype or torch.float32)


def test_binding_rejects_mis_sized_product_arguments():
    import torch
    X, V, th = _t(50, 3), _t(50, 4), _t(3, dtype=torch.float64)
    with pytest.raises(ValueError, match="rows"):
        gpk.kmatvec(X, th, _t(49, 4))
    with pytest.raises(ValueError, match="theta"):
        gpk.kmatvec(X, _t(4, dtype=torch.float64), V)
    with pytest.raises(ValueError, match="col_shift"):
        gpk.kmatvec(X, th, V, col_shift=_t(3, dtype=torch.float64))
    with pytest.raises(ValueError, match="out"):
        gpk.kmatvec(X, th, V, out=_t(50, 3))
    with pytest.raises(TypeError, match="out"):
        gpk.kmatvec(X, th, V, out=_t(50, 4, dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU"):
        gpk.kmatvec(X, th, V)
    with pytest.raises(ValueError, match="V has shape"):
        gpk.quadform_grad(X, th, V, _t(50, 3))
    with pytest.raises(ValueError, match="U has shape"):
        gpk.quadform_grad(X, th, _t(40, 4))
    with pytest.raises(ValueError, match="w has"):
        gpk.quadform_grad(X, th, V, V, _t(3, dtype=torch.float64))
    with pytest.raises(ValueError, match="theta"):
        gpk.quadform_grad(X, _t(4, dtype=torch.float64), V, kind="ard")
    with pytest.raises(ValueError, match="GPU"):
        gpk.quadform_grad(X, _t(5, dtype=torch.float64), V, kind="ard")
    with pytest.raises(ValueError, match="rows"):
        gpk.phi_refresh(X, th, _t(49, 1))
    with pytest.raises(ValueError, match="omega"):
        gpk.nystrom(X, th, _t(49, 5))
    with pytest.raises(ValueError, match="lam"):
        gpk.pcg_solve(X, th, _t(50, 2), U=_t(50, 5), lam=_t(4, dtype=torch.float64))
    with pytest.raises(ValueError, match="B has"):
        gpk.pcg_solve(X, th, _t(51, 2))


def test_binding_rejects_mis_sized_trajectory_arguments():
    import torch
    f64 = torch.float64
    ns, offs, chains = [30, 20], [0, 30], 3
    X, y = _t(50, 2), _t(50)
    phi, xw = _t(150), _t(150)
    th, pi, u = _t(18, dtype=f64), _t(18, dtype=f64), _t(6, dtype=f64)

    def call(**kw):
        a = dict(X=X, y=y, phi=phi, theta=th, pi=pi, x_warm=xw, u=u)
        a.update(kw)
        return gpk.hmc_leapfrog(a["X"], a["y"], a["phi"], a["theta"], a["pi"], a["x_warm"], "iso",
                                ns, offs, chains, u=a["u"])
    with pytest.raises(ValueError, match="GPU"):
        call()
    for name, bad in (("X", _t(49, 2)), ("y", _t(49)), ("phi", _t(149)), ("x_warm", _t(149)),
                      ("theta", _t(17, dtype=f64)), ("pi", _t(17, dtype=f64)), ("u", _t(5, dtype=f64))):
        with pytest.raises(ValueError, match=name):
            call(**{name: bad})
    with pytest.raises(ValueError, match="xi"):
        gpk.rwm(X, y, phi, th, _t(10, dtype=f64), xw, "iso", ns, offs, chains)
    with pytest.raises(ValueError, match="one entry per instance"):
        gpk.hmc_leapfrog(X, y, phi, th, pi, xw, "iso", ns, [0], chains)
    with pytest.raises(ValueError, match="pi"):
        gpk.hmc_implicit(X, y[:50], phi[:50], _t(3, dtype=f64), _t(2, dtype=f64), xw[:50])


def test_binding_rejects_mis_sized_refresh_arguments():
    import torch
    f64 = torch.float64
    ns, offs, chains = [30, 20], [0, 30], 3
    X, xi, th = _t(50, 2), _t(150), _t(18, dtype=f64)

    def call(**kw):
        a = dict(X=X, xi=xi, theta=th, out=None)
        a.update(kw)
        return gpk.phi_refresh_chains(a["X"], a["theta"], a["xi"], "iso", ns, offs, chains,
                                      out=a["out"])
    with pytest.raises(ValueError, match="GPU"):
        call()
    for name, bad in (("X", _t(49, 2)), ("xi", _t(149)), ("theta", _t(17, dtype=f64)),
                      ("out", _t(149))):
        with pytest.raises(ValueError, match=name):
            call(**{name: bad})
    with pytest.raises(TypeError, match="theta"):
        call(theta=_t(18))
    with pytest.raises(TypeError, match="out"):
        call(out=_t(150, dtype=f64))


def test_kmatvec_noalloc_validates_before_any_hip_call():
    # argument errors and a workspace that cannot fit the library's 64 MiB array are reported
    # with no HIP call (so this runs on a CPU-only host); empty products succeed
    L = gpk.lib()
    vp = ctypes.c_void_p

    def call(k, n, r=16, X=1 << 40, V=3 << 40, out=4 << 40):
        return L.gp_kmatvec_noalloc(k, n, vp(X), vp(2 << 40), r, vp(V), r, None, vp(out), r, None)
    iso32 = ctypes.byref(gpk.Kernel(gpk.ISO, gpk.F32, 3, 0))
    assert call(None, 10) == 1
    assert call(iso32, 10, X=0) == 1
    assert call(iso32, 10, V=4 << 40, out=4 << 40) == 1
    assert call(iso32, 400000) == 4
    assert b"limit" in L.gp_last_error()
    assert call(ctypes.byref(gpk.Kernel(gpk.ARD, gpk.BF16X, 64, 0)), 60000, r=1) == 4
    assert call(iso32, 0) == 0 and call(iso32, 10, r=0) == 0
