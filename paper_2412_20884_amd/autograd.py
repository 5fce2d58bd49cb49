"""torch.autograd Functions over libgpk with hand-written backward passes.

KMatVec.apply(X, theta, V, kind)   -> A(theta) V
    backward(G): one gp_quadform_grad pass with U = G, V = V gives
        dL/dtheta = sum_c G_c^T (dA/dtheta) V_c     and   dL/dV = A G   (A is symmetric)
QuadForm.apply(X, theta, U, V, kind) -> q, q_c = u_c^T A(theta) v_c
    forward keeps A V (O(N R), not the kernel matrix); backward(g): one pass with weights g gives
        dL/dtheta = sum_c g_c dq_c/dtheta,  dL/dV = (A U) diag(g)  and  dL/dU = (A V) diag(g).
Kernel tiles are recomputed in every pass, never stored.  X receives no gradient.
"""
from __future__ import annotations

import torch

from . import gpk

_MAX_R = 32


def _chunks(r):
    return [(c, min(r, c + _MAX_R)) for c in range(0, r, _MAX_R)]


class KMatVec(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, theta, V, kind="iso", n_cheb=0):
        ctx.kind = kind
        ctx.n_cheb = n_cheb
        ctx.save_for_backward(X, theta, V)
        return gpk.kmatvec(X, theta, V.contiguous(), kind, n_cheb=n_cheb)

    @staticmethod
    def backward(ctx, G):
        X, theta, V = ctx.saved_tensors
        need_t, need_v = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        if not (need_t or need_v):
            return None, None, None, None, None
        G = G.contiguous()
        V = V.contiguous()
        squeeze = V.dim() == 1
        G2 = G[:, None] if squeeze else G
        V2 = V[:, None] if squeeze else V
        dtheta = torch.zeros_like(theta) if need_t else None
        dV = torch.empty_like(V2) if need_v else None
        for c0, c1 in _chunks(V2.shape[1]):
            res = gpk.quadform_grad(X, theta, G2[:, c0:c1].contiguous(), V2[:, c0:c1].contiguous(), None,
                                    ctx.kind, want_grad=need_t, want_quad=False, want_AU=need_v,
                                    n_cheb=ctx.n_cheb)
            if need_t:
                dtheta += res["grad"]
            if need_v:
                dV[:, c0:c1] = res["AU"]
        if need_v and squeeze:
            dV = dV[:, 0]
        return None, dtheta, dV, None, None


class QuadForm(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, theta, U, V, kind="iso", n_cheb=0):
        if U.shape[1] > _MAX_R:
            raise ValueError("QuadForm takes at most 32 columns")
        U = U.contiguous()
        V = V.contiguous()
        res = gpk.quadform_grad(X, theta, U, V, None, kind, want_grad=False, want_quad=True, want_AV=True,
                                n_cheb=n_cheb)
        ctx.kind = kind
        ctx.n_cheb = n_cheb
        ctx.save_for_backward(X, theta, U, V, res["AV"])
        return res["quad"]

    @staticmethod
    def backward(ctx, g):
        X, theta, U, V, AV = ctx.saved_tensors
        need_t, need_u, need_v = ctx.needs_input_grad[1], ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        if not (need_t or need_u or need_v):
            return None, None, None, None, None, None
        g = g.contiguous().to(torch.float64)
        res = gpk.quadform_grad(X, theta, U, V, g, ctx.kind, want_grad=need_t, want_quad=not need_t,
                                want_AU=need_v, n_cheb=ctx.n_cheb)
        gd = g.to(U.dtype)[None, :]
        dU = AV * gd if need_u else None
        dV = res["AU"] * gd if need_v else None
        return None, res["grad"] if need_t else None, dU, dV, None, None


def kmatvec(X, theta, V, kind="iso", n_cheb=0):
    return KMatVec.apply(X, theta, V, kind, n_cheb)


def quadform(X, theta, U, V=None, kind="iso", n_cheb=0):
    return QuadForm.apply(X, theta, U, U if V is None else V, kind, n_cheb)
