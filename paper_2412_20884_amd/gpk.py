"""ctypes binding of libgpk (include/gpk.h): argument marshalling only.

Every computation runs in the library's HIP kernels; this module checks tensor placement,
dtype and layout, allocates the workspace and output tensors with PyTorch (device memory and
streams are the only things PyTorch provides here) and calls the C entry points on the current
stream.  The library is loaded on first use; if it has not been built the call fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgpk.so")

ISO, ARD, CHEB = 0, 1, 2
F64, F32, BF16X = 0, 1, 2
NO_NOISE = 1
PLAIN, BATCHED, GRAPH = 0, 1, 2
CHAIN_CG_MAXIT, CHAIN_NONFINITE_H, CHAIN_NONFINITE_THETA, CHAIN_ABORTED, CHAIN_FP_MAXIT = 1, 2, 4, 8, 16
PHI_CG_MAXIT, PHI_NONFINITE, PHI_ABORTED = 1, 2, 4
CG_MAXIT, CG_NONFINITE = 1, 2

EXPORTED = (
    "gp_last_error", "gp_status_string", "gp_n_theta", "gp_workspace_size", "gp_kmatvec",
    "gp_quadform_grad", "gp_hmc_workspace_size", "gp_hmc_leapfrog", "gp_tune_workspace_size",
    "gp_tune_products", "gp_tune_save", "gp_tune_load", "gp_tune_entries", "gp_tune_clear",
    "gp_pole_weights", "gp_phi_workspace_size", "gp_phi_refresh", "gp_nystrom_workspace_size",
    "gp_nystrom", "gp_pcg_workspace_size", "gp_pcg_solve", "gp_implicit_workspace_size",
    "gp_hmc_implicit", "gp_rwm", "gp_kmatvec_noalloc", "gp_tune_hmc_workspace_size", "gp_tune_hmc",
    "gp_phi_chains_workspace_size", "gp_phi_refresh_chains",
)


class GpkError(RuntimeError):
    def __init__(self, status, name, message):
        super().__init__(f"{name}: {message}")
        self.status = status


class Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("prec", ctypes.c_int32), ("d", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("n_cheb", ctypes.c_int32)]


class HmcParams(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("dt", ctypes.c_double), ("cg_tol", ctypes.c_double),
                ("cg_maxit", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("inv_mass", ctypes.POINTER(ctypes.c_double)), ("precond_rank", ctypes.c_int32),
                ("precond_U", ctypes.c_void_p), ("precond_lam", ctypes.c_void_p),
                ("progress", ctypes.c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("chains_per_inst", ctypes.c_int32),
                ("n_points", ctypes.POINTER(ctypes.c_int64)), ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("d", ctypes.POINTER(ctypes.c_int32)), ("x_offsets", ctypes.POINTER(ctypes.c_int64))]


class ImplicitParams(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("dt", ctypes.c_double), ("history", ctypes.c_int32),
                ("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("cg_tol", ctypes.c_double),
                ("cg_maxit", ctypes.c_int32), ("power_its", ctypes.c_int32)]


class PhiParams(ctypes.Structure):
    _fields_ = [("n_poles", ctypes.c_int32), ("tol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("lambda_max", ctypes.c_double), ("precond_rank", ctypes.c_int32),
                ("precond_U", ctypes.c_void_p), ("precond_lam", ctypes.c_void_p)]


_LIB = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t


def lib():
    """The loaded libgpk (loads it on first call; raises if it is not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python -m paper_2412_20884_amd.csrc.build")
    L = ctypes.CDLL(LIB_PATH)
    L.gp_last_error.restype = ctypes.c_char_p
    L.gp_last_error.argtypes = []
    L.gp_status_string.restype = ctypes.c_char_p
    L.gp_status_string.argtypes = [_i32]
    L.gp_n_theta.restype = _i32
    L.gp_n_theta.argtypes = [ctypes.POINTER(Kernel)]
    L.gp_workspace_size.restype = _sz
    L.gp_workspace_size.argtypes = [ctypes.POINTER(Kernel), _i64, _i32]
    L.gp_kmatvec.restype = _i32
    L.gp_kmatvec.argtypes = [ctypes.POINTER(Kernel), _i64, _vp, _vp, _i32, _vp, _i64, _vp, _vp,
                             _i64, _vp, _sz, _vp]
    L.gp_kmatvec_noalloc.restype = _i32
    L.gp_kmatvec_noalloc.argtypes = [ctypes.POINTER(Kernel), _i64, _vp, _vp, _i32, _vp, _i64, _vp,
                                     _vp, _i64, _vp]
    L.gp_quadform_grad.restype = _i32
    L.gp_quadform_grad.argtypes = [ctypes.POINTER(Kernel), _i64, _vp, _vp, _i32, _vp, _i64, _vp,
                                   _i64, _vp, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _sz, _vp]
    L.gp_hmc_workspace_size.restype = _sz
    L.gp_hmc_workspace_size.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(HmcParams),
                                        ctypes.POINTER(Batch)]
    L.gp_hmc_leapfrog.restype = _i32
    L.gp_hmc_leapfrog.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(HmcParams),
                                  ctypes.POINTER(Batch), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    L.gp_rwm.restype = _i32
    L.gp_rwm.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(HmcParams),
                                  ctypes.POINTER(Batch), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    L.gp_tune_workspace_size.restype = _sz
    L.gp_tune_workspace_size.argtypes = [ctypes.POINTER(Kernel), _i64, _i32]
    L.gp_tune_products.restype = _i32
    L.gp_tune_products.argtypes = [ctypes.POINTER(Kernel), _i64, _i32, _i32, _vp, _sz, _vp]
    L.gp_tune_hmc_workspace_size.restype = _sz
    L.gp_tune_hmc_workspace_size.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(HmcParams),
                                             ctypes.POINTER(Batch)]
    L.gp_tune_hmc.restype = _i32
    L.gp_tune_hmc.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(HmcParams),
                              ctypes.POINTER(Batch), _vp, _sz, _vp]
    L.gp_tune_save.restype = _i32
    L.gp_tune_save.argtypes = [ctypes.c_char_p]
    L.gp_tune_load.restype = _i32
    L.gp_tune_load.argtypes = [ctypes.c_char_p]
    L.gp_tune_entries.restype = _i32
    L.gp_tune_entries.argtypes = []
    L.gp_tune_clear.restype = None
    L.gp_tune_clear.argtypes = []
    L.gp_pole_weights.restype = _i32
    L.gp_pole_weights.argtypes = [ctypes.c_double, ctypes.c_double, _i32, _vp, _vp]
    L.gp_phi_workspace_size.restype = _sz
    L.gp_phi_workspace_size.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(PhiParams), _i64, _i32]
    L.gp_phi_refresh.restype = _i32
    L.gp_phi_refresh.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(PhiParams), _i64, _vp, _vp,
                                 _i32, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp]
    L.gp_phi_chains_workspace_size.restype = _sz
    L.gp_phi_chains_workspace_size.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(PhiParams),
                                               _i32, ctypes.POINTER(Batch)]
    L.gp_phi_refresh_chains.restype = _i32
    L.gp_phi_refresh_chains.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(PhiParams), _i32,
                                        ctypes.POINTER(Batch), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                        _vp, _sz, _vp]
    L.gp_nystrom_workspace_size.restype = _sz
    L.gp_nystrom_workspace_size.argtypes = [ctypes.POINTER(Kernel), _i64, _i32]
    L.gp_nystrom.restype = _i32
    L.gp_nystrom.argtypes = [ctypes.POINTER(Kernel), _i64, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp]
    L.gp_pcg_workspace_size.restype = _sz
    L.gp_pcg_workspace_size.argtypes = [ctypes.POINTER(Kernel), _i64, _i32, _i32]
    L.gp_pcg_solve.restype = _i32
    L.gp_pcg_solve.argtypes = [ctypes.POINTER(Kernel), _i64, _vp, _vp, _i32, _vp, _i64, _vp, _i64, _vp,
                               _i32, _vp, _vp, ctypes.c_double, _i32, _vp, _vp, _vp, _sz, _vp]
    L.gp_implicit_workspace_size.restype = _sz
    L.gp_implicit_workspace_size.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(ImplicitParams), _i64, _i32]
    L.gp_hmc_implicit.restype = _i32
    L.gp_hmc_implicit.argtypes = [ctypes.POINTER(Kernel), ctypes.POINTER(ImplicitParams), _i64, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    _LIB = L
    return L


def _check(status):
    if status != 0:
        L = lib()
        raise GpkError(status, L.gp_status_string(status).decode(), L.gp_last_error().decode())


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def kind_code(kind):
    if kind in (ISO, "iso"):
        return ISO
    if kind in (ARD, "ard"):
        return ARD
    if kind in (CHEB, "cheb"):
        return CHEB
    raise ValueError(f"unknown kernel kind {kind!r}")


def prec_code(dtype, prec=None):
    if prec in ("bf16x", BF16X):
        if dtype != torch.float32:
            raise TypeError("bf16x takes float32 tensors")
        return BF16X
    if dtype == torch.float64:
        return F64
    if dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {dtype}")


def make_kernel(kind, X, prec=None, no_noise=False, n_cheb=0):
    """Kernel description for points X; the Chebyshev-amplitude kernel ("cheb") needs n_cheb."""
    kc = kind_code(kind)
    if kc == CHEB and n_cheb < 1:
        raise ValueError("the Chebyshev-amplitude kernel needs n_cheb >= 1")
    return Kernel(kc, prec_code(X.dtype, prec), X.shape[1], NO_NOISE if no_noise else 0,
                  int(n_cheb))


def n_theta(kind, d, n_cheb=0):
    kc = kind_code(kind)
    if kc == CHEB:
        return int(n_cheb) ** d + 2
    return 3 if kc == ISO else d + 2


def _rowmajor(t, name):
    # strides of size-1 dimensions carry no meaning (torch may report any value for them)
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1) or \
            (t.shape[0] > 1 and t.stride(0) < t.shape[1]):
        raise ValueError(f"{name} must be a 2-D tensor with unit column stride")


def _same(device, dtype, **ts):
    for name, t in ts.items():
        if t is None:
            continue
        if t.device != device:
            raise ValueError(f"{name} is on {t.device}, expected {device}")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")


def _len_at_least(t, need, name):
    if t is not None and t.numel() < need:
        raise ValueError(f"{name} has {t.numel()} elements, at least {need} are needed")


def _exact_len(t, need, name):
    if t is not None and t.numel() != need:
        raise ValueError(f"{name} has {t.numel()} elements, expected {need}")


def _shape2(t, rows, cols, name):
    if t is not None and (t.dim() != 2 or t.shape[0] != rows or t.shape[1] != cols):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected ({rows}, {cols})")


def _on_gpu(*ts):
    # checked after every shape check, so that a mis-sized tensor is reported as such
    for t in ts:
        if t is not None and t.device.type != "cuda":
            raise ValueError(f"tensors must be on a GPU device, got {t.device}")


def workspace_size(kernel, n, r):
    return int(lib().gp_workspace_size(ctypes.byref(kernel), int(n), int(r)))


def _workspace(nbytes, device, ws=None):
    if nbytes == 0:
        return None
    if ws is not None and ws.numel() >= nbytes:
        return ws
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def kmatvec(X, theta, V, kind="iso", prec=None, col_shift=None, no_noise=False, out=None, ws=None,
            n_cheb=0):
    """(A(theta) + diag(col_shift)) V through gp_kmatvec.  V may be 1-D (one column)."""
    squeeze = V.dim() == 1
    V2 = V[:, None] if squeeze else V
    _rowmajor(X, "X")
    _rowmajor(V2, "V")
    if X.stride(0) != X.shape[1]:
        raise ValueError("X must be contiguous")
    dev = X.device
    _same(dev, X.dtype, V=V2)
    _same(dev, torch.float64, theta=theta, col_shift=col_shift)
    k = make_kernel(kind, X, prec, no_noise, n_cheb)
    n, r = X.shape[0], V2.shape[1]
    if V2.shape[0] != n:
        raise ValueError(f"V has {V2.shape[0]} rows, X has {n}")
    _exact_len(theta, n_theta(kind, X.shape[1], n_cheb), "theta")
    _exact_len(col_shift, r, "col_shift")
    if out is None:
        out = torch.empty((n, r), dtype=X.dtype, device=dev)
    out2 = out[:, None] if out.dim() == 1 else out
    _same(dev, X.dtype, out=out2)
    _shape2(out2, n, r, "out")
    _rowmajor(out2, "out")
    _on_gpu(X, V2, theta, col_shift, out2)
    w = _workspace(workspace_size(k, n, r), dev, ws)
    _check(lib().gp_kmatvec(ctypes.byref(k), n, _p(X), _p(theta), r, _p(V2), V2.stride(0),
                            _p(col_shift), _p(out2), out2.stride(0), _p(w),
                            0 if w is None else w.numel(), _stream(dev)))
    return out2[:, 0] if squeeze else out


def quadform_grad(X, theta, U, V=None, w=None, kind="iso", prec=None, want_grad=True,
                  want_quad=True, want_AU=False, want_AV=False, ws=None, n_cheb=0, no_noise=False):
    """sum_c w_c u_c^T A v_c: dict with 'grad' (n_theta), 'quad' (R), 'AU', 'AV' as requested."""
    if V is None:
        V = U
    _rowmajor(X, "X")
    _rowmajor(U, "U")
    _rowmajor(V, "V")
    dev = X.device
    _same(dev, X.dtype, U=U, V=V)
    _same(dev, torch.float64, theta=theta, w=w)
    k = make_kernel(kind, X, prec, no_noise, n_cheb)
    n, r = X.shape[0], U.shape[1]
    nt = n_theta(kind, X.shape[1], n_cheb)
    _shape2(U, n, r, "U")
    _shape2(V, n, r, "V")
    _exact_len(theta, nt, "theta")
    _exact_len(w, r, "w")
    _on_gpu(X, U, V, theta, w)
    grad = torch.empty(nt, dtype=torch.float64, device=dev) if want_grad else None
    quad = torch.empty(r, dtype=torch.float64, device=dev) if want_quad else None
    AU = torch.empty((n, r), dtype=X.dtype, device=dev) if want_AU else None
    AV = torch.empty((n, r), dtype=X.dtype, device=dev) if want_AV else None
    wk = _workspace(workspace_size(k, n, r), dev, ws)
    _check(lib().gp_quadform_grad(ctypes.byref(k), n, _p(X), _p(theta), r, _p(U), U.stride(0),
                                  _p(V), V.stride(0), _p(w), _p(grad), _p(quad), _p(AU),
                                  r, _p(AV), r, _p(wk), 0 if wk is None else wk.numel(),
                                  _stream(dev)))
    return {"grad": grad, "quad": quad, "AU": AU, "AV": AV}


_HMC_WS = {}


def _check_batch(X, y, phi, theta, pi, x_warm, u, kind, n_points, offsets, chains, dims,
                 x_offsets, n_cheb, pi_name="pi", phi_name="phi", xw_name="x_warm"):
    """Lengths of the packed arrays against the batch description (packing of include/gpk.h)."""
    n_inst = len(n_points)
    if n_inst < 1 or len(offsets) != n_inst or len(dims) != n_inst:
        raise ValueError("n_points, offsets and d must have one entry per instance")
    if x_offsets is not None and len(x_offsets) != n_inst:
        raise ValueError("x_offsets must have one entry per instance")
    if int(chains) < 1:
        raise ValueError("chains must be >= 1")
    need_x = need_y = need_v = 0
    nth_total = 0
    for b in range(n_inst):
        nb, ob, db = int(n_points[b]), int(offsets[b]), int(dims[b])
        if nb < 1 or ob < 0:
            raise ValueError(f"instance {b}: n_points must be >= 1 and offsets >= 0")
        xo = ob * db if x_offsets is None else int(x_offsets[b])
        need_x = max(need_x, xo + nb * db)
        need_y = max(need_y, ob + nb)
        need_v = max(need_v, int(chains) * (ob + nb))
        nth_total += n_theta(kind, db, n_cheb)
    _len_at_least(X, need_x, "X")
    _len_at_least(y, need_y, "y")
    _len_at_least(phi, need_v, phi_name)
    _len_at_least(x_warm, need_v, xw_name)
    _len_at_least(theta, int(chains) * nth_total, "theta")
    _len_at_least(pi, int(chains) * nth_total, pi_name)
    _len_at_least(u, n_inst * int(chains), "u")
    _on_gpu(X, y, phi, theta, pi, x_warm, u)
    return nth_total


def _chain_outputs(outputs, names, nc, dev, cg_iters):
    """Per-chain output tensors: the caller's (a dict from an earlier call, so that graph mode
    replays with unchanged descriptors) or new ones."""
    if outputs is not None:
        o = outputs
        for key, dt in ((names[0], torch.float64), (names[1], torch.float64),
                        ("accepted", torch.int32), ("status", torch.int32)):
            t = o[key]
            if t.dtype != dt or t.numel() != nc or t.device != dev or not t.is_contiguous():
                raise ValueError(f"outputs[{key!r}] must be a contiguous {dt} tensor of {nc} on {dev}")
        it = o.get("cg_iters")
        if it is not None and (it.dtype != torch.int32 or it.numel() != nc or it.device != dev):
            raise ValueError("outputs['cg_iters'] must be an int32 tensor of one entry per chain")
        return o[names[0]], o[names[1]], o["accepted"], o["status"], it
    return (torch.empty(nc, dtype=torch.float64, device=dev),
            torch.empty(nc, dtype=torch.float64, device=dev),
            torch.empty(nc, dtype=torch.int32, device=dev),
            torch.empty(nc, dtype=torch.int32, device=dev),
            torch.empty(nc, dtype=torch.int32, device=dev) if cg_iters else None)


def _hmc_params(n_steps, dt, cg_tol, cg_maxit, mode, inv_mass, precond, nth_total, n_points,
                offsets, X, progress=None):
    """gp_hmc_params; inv_mass: host sequence (one instance's n_theta, or all instances' packed),
    precond: (U, lam) tensors packed per instance (gp_hmc_params in include/gpk.h), or None.
    Returns (params, keep-alive objects)."""
    keep = []
    im = None
    if inv_mass is not None:
        vals = [float(v) for v in (inv_mass.tolist() if hasattr(inv_mass, "tolist") else inv_mass)]
        if len(vals) != nth_total:
            raise ValueError(f"inv_mass has {len(vals)} entries, the batch has {nth_total}")
        im = (ctypes.c_double * nth_total)(*vals)
        keep.append(im)
    rank, pU, plam = 0, None, None
    if precond is not None:
        U, lam = precond
        if U.dim() != 2 or not U.is_contiguous() or not lam.is_contiguous():
            raise ValueError("precond U must be a contiguous 2-D tensor (rows x rank)")
        rank = U.shape[1]
        _same(X.device, X.dtype, precond_U=U)
        _same(X.device, torch.float64, precond_lam=lam)
        need_u = max(int(o) + int(n) for o, n in zip(offsets, n_points))
        _len_at_least(U, need_u * rank, "precond U")
        _len_at_least(lam, len(n_points) * rank, "precond lam")
        _on_gpu(U, lam)
        pU, plam = _p(U), _p(lam)
    if progress is not None and (progress.dtype != torch.int32 or progress.numel() < 1 or
                                 not (progress.is_cuda or progress.is_pinned())):
        raise ValueError("progress must be a pinned host or device int32 tensor")
    prm = HmcParams(int(n_steps), float(dt), float(cg_tol), int(cg_maxit), int(mode),
                    ctypes.cast(im, ctypes.POINTER(ctypes.c_double)) if im is not None else None,
                    int(rank), pU, plam, _p(progress))
    return prm, keep


def hmc_workspace_size(kernel, params, batch):
    return int(lib().gp_hmc_workspace_size(ctypes.byref(kernel), ctypes.byref(params), ctypes.byref(batch)))


def hmc_leapfrog(X, y, phi, theta, pi, x_warm, kind, n_points, offsets, chains, d=None,
                 x_offsets=None, u=None, n_steps=20, dt=1e-2, cg_tol=1e-6, cg_maxit=1000,
                 mode=BATCHED, ws=None, cg_iters=True, prec=None, n_cheb=0, inv_mass=None,
                 precond=None, outputs=None, progress=None):
    """One HMC trajectory per chain through gp_hmc_leapfrog (packing as in include/gpk.h).

    inv_mass: host sequence, the diagonal of M^{-1} packed per instance (None: M = I; a zero
    entry holds that hyperparameter fixed).  precond: (U, lam), a Nystrom factor per instance
    packed as in gp_hmc_params, with which every solve is preconditioned (None: plain CG).
    outputs: the dict an earlier call returned, to be written again (graph mode then replays its
    captured launch without a new capture).  progress: a pinned host (or device) int32 tensor into
    which the batched scheduler writes the number of finished chains while it runs.

    theta, pi and x_warm are updated in place.  Returns dict(H0, H1, accepted, status, cg_iters).
    The workspace is kept per (device, size) so repeated calls reuse it (and a captured graph).
    """
    dev = X.device
    dt_ = X.dtype
    _same(dev, dt_, y=y, phi=phi, x_warm=x_warm)
    _same(dev, torch.float64, theta=theta, pi=pi, u=u)
    for name, t in (("X", X), ("y", y), ("phi", phi), ("theta", theta), ("pi", pi), ("x_warm", x_warm)):
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    n_inst = len(n_points)
    dims = [X.shape[1]] * n_inst if d is None else list(d)
    nth_total = _check_batch(X, y, phi, theta, pi, x_warm, u, kind, n_points, offsets, chains,
                             dims, x_offsets, n_cheb)
    k = Kernel(kind_code(kind), prec_code(dt_, prec), int(max(dims)), 0, int(n_cheb))
    prm, _keep = _hmc_params(n_steps, dt, cg_tol, cg_maxit, mode, inv_mass, precond, nth_total,
                             n_points, offsets, X, progress)
    npts = (ctypes.c_int64 * n_inst)(*[int(v) for v in n_points])
    offs = (ctypes.c_int64 * n_inst)(*[int(v) for v in offsets])
    dd = (ctypes.c_int32 * n_inst)(*[int(v) for v in dims]) if d is not None else None
    xo = (ctypes.c_int64 * n_inst)(*[int(v) for v in x_offsets]) if x_offsets is not None else None
    b = Batch(n_inst, int(chains), npts, offs, dd, xo)
    nc = n_inst * chains
    H0, H1, acc, st, it = _chain_outputs(outputs, ("H0", "H1"), nc, dev, cg_iters)
    nbytes = hmc_workspace_size(k, prm, b)
    if nbytes == 0:
        _check(lib().gp_hmc_leapfrog(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b), None, None,
                                     None, None, None, None, None, None, None, None, None, None,
                                     None, 0, None))
    if ws is None:
        key = (str(dev), nbytes)
        ws = _HMC_WS.get(key)
        if ws is None:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            _HMC_WS[key] = ws
    _check(lib().gp_hmc_leapfrog(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b), _p(X), _p(y),
                                 _p(phi), _p(theta), _p(pi), _p(x_warm), _p(u), _p(H0), _p(H1),
                                 _p(acc), _p(st), _p(it), _p(ws), ws.numel(), _stream(dev)))
    return {"H0": H0, "H1": H1, "accepted": acc, "status": st, "cg_iters": it}


def rwm(X, y, phi, theta, xi, x_warm, kind, n_points, offsets, chains, d=None, x_offsets=None,
        u=None, dt=0.1, cg_tol=1e-6, cg_maxit=1000, mode=BATCHED, ws=None, cg_iters=True,
        prec=None, n_cheb=0, inv_mass=None, precond=None, outputs=None):
    """One random-walk Metropolis update per chain through gp_rwm (packing as in include/gpk.h):
    proposal theta + dt * xi, accepted when log u <= U0 - U1.

    theta and x_warm are updated in place.  Returns dict(U0, U1, accepted, status, cg_iters).
    """
    dev = X.device
    dt_ = X.dtype
    _same(dev, dt_, y=y, phi=phi, x_warm=x_warm)
    _same(dev, torch.float64, theta=theta, xi=xi, u=u)
    for name, t in (("X", X), ("y", y), ("phi", phi), ("theta", theta), ("xi", xi), ("x_warm", x_warm)):
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    n_inst = len(n_points)
    dims = [X.shape[1]] * n_inst if d is None else list(d)
    nth_total = _check_batch(X, y, phi, theta, xi, x_warm, u, kind, n_points, offsets, chains,
                             dims, x_offsets, n_cheb, pi_name="xi")
    k = Kernel(kind_code(kind), prec_code(dt_, prec), int(max(dims)), 0, int(n_cheb))
    prm, _keep = _hmc_params(0, dt, cg_tol, cg_maxit, mode, inv_mass, precond, nth_total,
                             n_points, offsets, X)
    npts = (ctypes.c_int64 * n_inst)(*[int(v) for v in n_points])
    offs = (ctypes.c_int64 * n_inst)(*[int(v) for v in offsets])
    dd = (ctypes.c_int32 * n_inst)(*[int(v) for v in dims]) if d is not None else None
    xo = (ctypes.c_int64 * n_inst)(*[int(v) for v in x_offsets]) if x_offsets is not None else None
    b = Batch(n_inst, int(chains), npts, offs, dd, xo)
    nc = n_inst * chains
    U0, U1, acc, st, it = _chain_outputs(outputs, ("U0", "U1"), nc, dev, cg_iters)
    nbytes = hmc_workspace_size(k, prm, b)
    if nbytes == 0:
        _check(lib().gp_rwm(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b), None, None, None,
                            None, None, None, None, None, None, None, None, None, None, 0, None))
    if ws is None:
        key = (str(dev), nbytes)
        ws = _HMC_WS.get(key)
        if ws is None:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            _HMC_WS[key] = ws
    _check(lib().gp_rwm(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b), _p(X), _p(y), _p(phi),
                        _p(theta), _p(xi), _p(x_warm), _p(u), _p(U0), _p(U1), _p(acc), _p(st),
                        _p(it), _p(ws), ws.numel(), _stream(dev)))
    return {"U0": U0, "U1": U1, "accepted": acc, "status": st, "cg_iters": it}


def tune(kind, d, n, r, dtype=torch.float32, with_grad=True, device="cuda:0", prec=None):
    """Autotune the product kernels for this problem class (synthetic inputs on `device`)."""
    k = Kernel(kind_code(kind), prec_code(dtype, prec), int(d), 0)
    nbytes = int(lib().gp_tune_workspace_size(ctypes.byref(k), int(n), int(r)))
    if nbytes == 0:
        raise ValueError("no product kernels for this description")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    _check(lib().gp_tune_products(ctypes.byref(k), int(n), int(r), 1 if with_grad else 0, _p(ws),
                                  nbytes, _stream(torch.device(device))))
    return int(lib().gp_tune_entries())


def tune_hmc(kind, n_points, chains, d, dtype=torch.float32, prec=None, n_cheb=0,
             precond_rank=0, device="cuda:0"):
    """Autotune the batched / graph trajectory launch for a batch of this geometry (instances of
    n_points[i] points in d[i] dimensions, `chains` chains each) on synthetic inputs.  Returns the
    number of entries in the tuning table."""
    n_points = [int(v) for v in n_points]
    dims = [int(v) for v in d]
    if len(dims) != len(n_points) or not n_points:
        raise ValueError("n_points and d need one entry per instance")
    k = Kernel(kind_code(kind), prec_code(dtype, prec), max(dims), 0, int(n_cheb))
    dev = torch.device(device)
    keep = []
    pU = plam = None
    if precond_rank:
        # the tuner reads no factor; any valid pointers satisfy the parameter check
        keep.append(torch.empty(1, dtype=torch.float64, device=dev))
        pU = plam = _p(keep[0])
    prm = HmcParams(1, 0.0, 1e-6, 4, BATCHED, None, int(precond_rank), pU, plam, None)
    npts = (ctypes.c_int64 * len(n_points))(*n_points)
    offs_l, o = [], 0
    for v in n_points:
        offs_l.append(o)
        o += v
    offs = (ctypes.c_int64 * len(n_points))(*offs_l)
    dd = (ctypes.c_int32 * len(dims))(*dims)
    b = Batch(len(n_points), int(chains), npts, offs, dd, None)
    nbytes = int(lib().gp_tune_hmc_workspace_size(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b)))
    if nbytes == 0:
        _check(lib().gp_tune_hmc(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b), None, 0, None))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    _check(lib().gp_tune_hmc(ctypes.byref(k), ctypes.byref(prm), ctypes.byref(b), _p(ws), nbytes,
                             _stream(dev)))
    return int(lib().gp_tune_entries())


def tune_save(path):
    _check(lib().gp_tune_save(str(path).encode()))


def tune_load(path):
    _check(lib().gp_tune_load(str(path).encode()))


def tune_entries():
    return int(lib().gp_tune_entries())


def tune_clear():
    lib().gp_tune_clear()


def pole_weights(m, M, n_poles=15):
    """(w, shifts) of the pole expansion of A^{-1/2} on [m, M], computed by the library (host)."""
    import numpy as np
    w = np.zeros(int(n_poles))
    sh = np.zeros(int(n_poles))
    _check(lib().gp_pole_weights(float(m), float(M), int(n_poles), w.ctypes.data_as(_vp),
                                 sh.ctypes.data_as(_vp)))
    return w, sh


def phi_workspace_size(kernel, params, n, r):
    return int(lib().gp_phi_workspace_size(ctypes.byref(kernel), ctypes.byref(params), int(n), int(r)))


_PHI_WS = {}


def phi_refresh_chains(X, theta, xi, kind, n_points, offsets, chains, d=None, x_offsets=None,
                       prec=None, n_poles=15, tol=1e-8, maxit=2000, lambda_max=None, mode=BATCHED,
                       out=None, ws=None, n_cheb=0, outputs=None):
    """phi_c = A(theta_c)^{-1/2} xi_c for every chain of a batch through gp_phi_refresh_chains
    (packing of gp_hmc_leapfrog: xi and phi as its phi, theta as its theta).  out: the phi tensor
    to write (may be xi itself; default a new one).  outputs: the dict an earlier call returned, to
    be written again (graph mode then replays its captured launches).

    Returns dict(phi, status, iters, bounds) with bounds one (m, M) row per chain."""
    dev = X.device
    dt_ = X.dtype
    _same(dev, dt_, xi=xi, out=out)
    _same(dev, torch.float64, theta=theta)
    for name, t in (("X", X), ("theta", theta), ("xi", xi), ("out", out)):
        if t is not None and not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    n_inst = len(n_points)
    dims = [X.shape[1]] * n_inst if d is None else list(d)
    _check_batch(X, None, xi, theta, None, out, None, kind, n_points, offsets, chains, dims,
                 x_offsets, n_cheb, phi_name="xi", xw_name="out")
    k = Kernel(kind_code(kind), prec_code(dt_, prec), int(max(dims)), 0, int(n_cheb))
    prm = PhiParams(int(n_poles), float(tol), int(maxit), float(lambda_max or 0.0), 0, None, None)
    npts = (ctypes.c_int64 * n_inst)(*[int(v) for v in n_points])
    offs = (ctypes.c_int64 * n_inst)(*[int(v) for v in offsets])
    dd = (ctypes.c_int32 * n_inst)(*[int(v) for v in dims]) if d is not None else None
    xo = (ctypes.c_int64 * n_inst)(*[int(v) for v in x_offsets]) if x_offsets is not None else None
    b = Batch(n_inst, int(chains), npts, offs, dd, xo)
    nc = n_inst * int(chains)
    if outputs is not None:
        st, it, bnd = outputs["status"], outputs["iters"], outputs["bounds"]
        for name, t, dt, m in (("status", st, torch.int32, nc), ("iters", it, torch.int32, nc),
                               ("bounds", bnd, torch.float64, 2 * nc)):
            if t.dtype != dt or t.numel() != m or t.device != dev or not t.is_contiguous():
                raise ValueError(f"outputs[{name!r}] must be a contiguous {dt} tensor of {m} on {dev}")
        if out is None:
            out = outputs["phi"]
    else:
        st = torch.zeros(nc, dtype=torch.int32, device=dev)
        it = torch.zeros(nc, dtype=torch.int32, device=dev)
        bnd = torch.zeros((nc, 2), dtype=torch.float64, device=dev)
    if out is None:
        out = torch.empty_like(xi)
    nbytes = int(lib().gp_phi_chains_workspace_size(ctypes.byref(k), ctypes.byref(prm), int(mode),
                                                    ctypes.byref(b)))
    if nbytes == 0:
        _check(lib().gp_phi_refresh_chains(ctypes.byref(k), ctypes.byref(prm), int(mode),
                                           ctypes.byref(b), None, None, None, None, None, None,
                                           None, None, 0, None))
    if ws is None:
        key = (str(dev), nbytes)
        ws = _PHI_WS.get(key)
        if ws is None:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            _PHI_WS[key] = ws
    _check(lib().gp_phi_refresh_chains(ctypes.byref(k), ctypes.byref(prm), int(mode), ctypes.byref(b),
                                       _p(X), _p(theta), _p(xi), _p(out), _p(st), _p(it), _p(bnd),
                                       _p(ws), ws.numel(), _stream(dev)))
    return {"phi": out, "status": st, "iters": it, "bounds": bnd}


def phi_refresh(X, theta, xi, kind="iso", prec=None, n_poles=15, tol=1e-8, maxit=2000,
                lambda_max=None, out=None, ws=None, n_cheb=0, precond=None):
    """phi = A(theta)^{-1/2} xi through gp_phi_refresh.  xi may be 1-D (one column).
    precond: (U, lam) from nystrom() to solve the shifted systems by preconditioned CG.

    Returns dict(phi, status, iters, bounds=(m, M))."""
    squeeze = xi.dim() == 1
    xi2 = xi[:, None] if squeeze else xi
    _rowmajor(X, "X")
    _rowmajor(xi2, "xi")
    if X.stride(0) != X.shape[1]:
        raise ValueError("X must be contiguous")
    dev = X.device
    _same(dev, X.dtype, xi=xi2)
    _same(dev, torch.float64, theta=theta)
    k = make_kernel(kind, X, prec, n_cheb=n_cheb)
    rank, pU, plam = 0, None, None
    if precond is not None:
        U, lam = precond
        _same(dev, X.dtype, precond_U=U)
        _same(dev, torch.float64, precond_lam=lam)
        if U.dim() != 2 or U.shape[0] != X.shape[0] or not U.is_contiguous():
            raise ValueError(f"precond U must be a contiguous {X.shape[0]} x rank tensor")
        _exact_len(lam, U.shape[1], "precond lam")
        _on_gpu(U, lam)
        rank, pU, plam = U.shape[1], _p(U), _p(lam)
    prm = PhiParams(int(n_poles), float(tol), int(maxit), float(lambda_max or 0.0), int(rank), pU,
                    plam)
    n, r = X.shape[0], xi2.shape[1]
    if xi2.shape[0] != n:
        raise ValueError(f"xi has {xi2.shape[0]} rows, X has {n}")
    _exact_len(theta, n_theta(kind, X.shape[1], n_cheb), "theta")
    if out is None:
        out = torch.empty((n, r), dtype=X.dtype, device=dev)
    out2 = out[:, None] if out.dim() == 1 else out
    _same(dev, X.dtype, out=out2)
    _shape2(out2, n, r, "out")
    _rowmajor(out2, "out")
    _on_gpu(X, theta, xi2, out2)
    status = torch.empty(r, dtype=torch.int32, device=dev)
    iters = torch.empty(r, dtype=torch.int32, device=dev)
    bounds = (ctypes.c_double * 2)(0.0, 0.0)
    w = _workspace(phi_workspace_size(k, prm, n, r), dev, ws)
    _check(lib().gp_phi_refresh(ctypes.byref(k), ctypes.byref(prm), n, _p(X), _p(theta), r,
                                _p(xi2), xi2.stride(0), _p(out2), out2.stride(0), _p(status),
                                _p(iters), ctypes.cast(bounds, _vp), _p(w),
                                0 if w is None else w.numel(), _stream(dev)))
    return {"phi": out2[:, 0] if squeeze else out, "status": status, "iters": iters,
            "bounds": (bounds[0], bounds[1])}


def nystrom(X, theta, omega, kind="iso", prec=None, n_cheb=0, ws=None):
    """Randomized Nystrom factor K ~ U diag(lam) U^T for the n x rank test matrix omega.
    Returns (U, lam)."""
    _rowmajor(X, "X")
    dev = X.device
    _same(dev, X.dtype, omega=omega)
    _same(dev, torch.float64, theta=theta)
    if not omega.is_contiguous():
        raise ValueError("omega must be contiguous")
    k = make_kernel(kind, X, prec, n_cheb=n_cheb)
    if omega.dim() != 2 or omega.shape[0] != X.shape[0]:
        raise ValueError(f"omega must be {X.shape[0]} x rank")
    _exact_len(theta, n_theta(kind, X.shape[1], n_cheb), "theta")
    _on_gpu(X, theta, omega)
    n, rank = omega.shape
    U = torch.empty((n, rank), dtype=X.dtype, device=dev)
    lam = torch.empty(rank, dtype=torch.float64, device=dev)
    nbytes = int(lib().gp_nystrom_workspace_size(ctypes.byref(k), n, rank))
    w = _workspace(nbytes, dev, ws)
    _check(lib().gp_nystrom(ctypes.byref(k), n, _p(X), _p(theta), rank, _p(omega), _p(U), _p(lam),
                            _p(w), 0 if w is None else w.numel(), _stream(dev)))
    return U, lam


def pcg_solve(X, theta, B, kind="iso", prec=None, x0=None, col_shift=None, U=None, lam=None,
              tol=1e-6, maxit=5000, n_cheb=0, ws=None):
    """(A + diag(col_shift)) x = B by (Nystrom-preconditioned if U is given) CG.  B may be 1-D.
    Returns dict(x, status, iters)."""
    squeeze = B.dim() == 1
    B2 = B[:, None] if squeeze else B
    _rowmajor(X, "X")
    _rowmajor(B2, "B")
    dev = X.device
    _same(dev, X.dtype, B=B2, U=U)
    _same(dev, torch.float64, theta=theta, col_shift=col_shift, lam=lam)
    k = make_kernel(kind, X, prec, n_cheb=n_cheb)
    n, r = B2.shape
    if n != X.shape[0]:
        raise ValueError(f"B has {n} rows, X has {X.shape[0]}")
    rank = 0 if U is None else U.shape[1]
    if U is not None and not U.is_contiguous():
        raise ValueError("U must be contiguous")
    if (U is None) != (lam is None):
        raise ValueError("U and lam go together")
    _shape2(U, n, rank, "U")
    _exact_len(lam, rank, "lam")
    _exact_len(theta, n_theta(kind, X.shape[1], n_cheb), "theta")
    _exact_len(col_shift, r, "col_shift")
    if x0 is not None:
        _shape2(x0[:, None] if x0.dim() == 1 else x0, n, r, "x0")
        _same(dev, X.dtype, x0=x0)
    _on_gpu(X, theta, B2, U, lam, col_shift, x0)
    x = torch.zeros((n, r), dtype=X.dtype, device=dev) if x0 is None else \
        (x0[:, None] if x0.dim() == 1 else x0).clone().contiguous()
    status = torch.empty(r, dtype=torch.int32, device=dev)
    iters = torch.empty(r, dtype=torch.int32, device=dev)
    nbytes = int(lib().gp_pcg_workspace_size(ctypes.byref(k), n, r, rank))
    w = _workspace(nbytes, dev, ws)
    _check(lib().gp_pcg_solve(ctypes.byref(k), n, _p(X), _p(theta), r, _p(B2), B2.stride(0), _p(x),
                              x.stride(0), _p(col_shift), rank, _p(U), _p(lam), float(tol), int(maxit),
                              _p(status), _p(iters), _p(w), 0 if w is None else w.numel(), _stream(dev)))
    return {"x": x[:, 0] if squeeze else x, "status": status, "iters": iters}


def hmc_implicit(X, y, phi, theta, pi, x_warm, kind="iso", n_steps=3, dt=0.1, history=10, tol=1e-10,
                 maxit=200, cg_tol=1e-6, cg_maxit=5000, power_its=10, u=None, U=None, lam=None,
                 prec=None, n_cheb=0, ws=None):
    """One implicit-midpoint HMC trajectory of one chain through gp_hmc_implicit.

    theta, pi and x_warm are updated in place.  Returns dict(H0, H1, accepted, status, iters)."""
    _rowmajor(X, "X")
    dev = X.device
    _same(dev, X.dtype, y=y, phi=phi, x_warm=x_warm, U=U)
    _same(dev, torch.float64, theta=theta, pi=pi, u=u, lam=lam)
    for name, t in (("y", y), ("phi", phi), ("theta", theta), ("pi", pi), ("x_warm", x_warm)):
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    k = make_kernel(kind, X, prec, n_cheb=n_cheb)
    n = X.shape[0]
    nt = n_theta(kind, X.shape[1], n_cheb)
    for name, t, m in (("y", y, n), ("phi", phi, n), ("x_warm", x_warm, n), ("theta", theta, nt),
                       ("pi", pi, nt)):
        _exact_len(t, m, name)
    _len_at_least(u, 1, "u")
    if (U is None) != (lam is None):
        raise ValueError("U and lam go together")
    if U is not None:
        if U.dim() != 2 or U.shape[0] != n or not U.is_contiguous():
            raise ValueError(f"U must be a contiguous {n} x rank tensor")
        _exact_len(lam, U.shape[1], "lam")
    _on_gpu(X, y, phi, theta, pi, x_warm, u, U, lam)
    prm = ImplicitParams(int(n_steps), float(dt), int(history), float(tol), int(maxit), float(cg_tol),
                         int(cg_maxit), int(power_its))
    n = X.shape[0]
    rank = 0 if U is None else U.shape[1]
    out = {key: torch.empty(1, dtype=torch.float64, device=dev) for key in ("H0", "H1")}
    out.update({key: torch.empty(1, dtype=torch.int32, device=dev) for key in ("accepted", "status", "iters")})
    nbytes = int(lib().gp_implicit_workspace_size(ctypes.byref(k), ctypes.byref(prm), n, rank))
    w = _workspace(nbytes, dev, ws)
    _check(lib().gp_hmc_implicit(ctypes.byref(k), ctypes.byref(prm), n, _p(X), _p(y), _p(phi), _p(theta),
                                 _p(pi), _p(x_warm), _p(u), rank, _p(U), _p(lam), _p(out["H0"]),
                                 _p(out["H1"]), _p(out["accepted"]), _p(out["status"]), _p(out["iters"]),
                                 _p(w), 0 if w is None else w.numel(), _stream(dev)))
    return out
