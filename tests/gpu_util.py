"""Helpers for the GPU parity tests: device placement and error metrics against the oracle."""
import numpy as np
import torch

DEV = "cuda:0"


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rounded(a, dtype):
    """The values a device array of `dtype` holds, as float64 on the host (the oracle's input)."""
    if dtype == torch.float64:
        return np.asarray(a, dtype=np.float64)
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def col_rel_err(out, ref):
    """max_c |out_c - ref_c|_2 / |ref_c|_2."""
    out = np.atleast_2d(out.T).T if out.ndim == 1 else out
    ref = np.atleast_2d(ref.T).T if ref.ndim == 1 else ref
    num = np.linalg.norm(out - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return float(np.max(num / np.maximum(den, 1e-300)))


def grad_rel_err(g, ref, scale):
    """max_p |g_p - ref_p| / scale_p, scale_p = sum_c |w_c| |u_c|^T |dA/dtheta_p| |v_c|."""
    return float(np.max(np.abs(g - ref) / np.maximum(scale, 1e-300)))


def comp_rel_err(out, ref, absref):
    """max_ic |out_ic - ref_ic| / (|A| |V|)_ic: the componentwise, condition-aware error (absref is
    the oracle's product with |V|; every entry of A is positive, so |A| |V| = A |V|)."""
    out = out.reshape(ref.shape)
    return float(np.max(np.abs(out - ref) / np.maximum(absref, 1e-300)))
