"""torch.autograd.Function for the weighted smoothed cost h_{mu,w}(x - U y)
(Sec. 3.1, eqs. weightedLPnorm / spcacost) over a batch of frames.

Forward and backward are the HIP kernels behind pros_lpcost_fwd /
pros_lpcost_bwd; this module only allocates outputs and workspace with torch
and passes pointers and the current stream.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L

_COST = {"lp": L.PROS_COST_LP, "log": L.PROS_COST_LOG}


def _sig():
    return L.lib()


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_inputs(U, Y, X, mu, w):
    for name, t in (("U", U), ("Y", Y), ("X", X), ("mu", mu)):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float32 GPU tensor")
    m, k = U.shape
    B = Y.shape[0]
    if Y.shape != (B, k) or X.shape != (B, m) or mu.numel() != 1:
        raise ValueError(f"shapes U{tuple(U.shape)} Y{tuple(Y.shape)} X{tuple(X.shape)} mu{tuple(mu.shape)}")
    if w is not None and (w.shape != (m,) or w.dtype != torch.float32 or not w.is_cuda or not w.is_contiguous()):
        raise ValueError("w must be a contiguous float32 GPU tensor of shape (m,)")
    return m, k, B


def _workspace(m, k, B, device):
    n = _sig().pros_lpcost_workspace_size(m, k, B)
    return torch.empty(n, dtype=torch.uint8, device=device), n


class LpCost(torch.autograd.Function):
    """f[b] = sum_e w_e phi(X[b,e] - U[e,:] . Y[b,:]); gradients for U, Y, X, mu."""

    @staticmethod
    def forward(ctx, U, Y, X, mu, w=None, p=0.25, cost="lp"):
        m, k, B = _check_inputs(U, Y, X, mu, w)
        lib = _sig()
        ws, nws = _workspace(m, k, B, U.device)
        f = torch.empty(B, dtype=torch.float32, device=U.device)
        st = torch.cuda.current_stream().cuda_stream
        L.check(lib.pros_lpcost_fwd(_p(U), _p(Y), _p(X), _p(w), _p(mu), m, k, B, _COST[cost], float(p),
                                    _p(f), _p(ws), nws, C.c_void_p(st)))
        ctx.save_for_backward(U, Y, X, mu, w)
        ctx.p, ctx.cost = float(p), cost
        return f

    @staticmethod
    def backward(ctx, gout):
        U, Y, X, mu, w = ctx.saved_tensors
        m, k = U.shape
        B = Y.shape[0]
        lib = _sig()
        gout = gout.contiguous().to(torch.float32)
        need = ctx.needs_input_grad
        dU = torch.empty_like(U) if need[0] else None
        dY = torch.empty_like(Y) if need[1] else None
        dX = torch.empty_like(X) if need[2] else None
        dmu = torch.empty(1, dtype=torch.float32, device=U.device) if need[3] else None
        ws, nws = _workspace(m, k, B, U.device)
        st = torch.cuda.current_stream().cuda_stream
        L.check(lib.pros_lpcost_bwd(_p(U), _p(Y), _p(X), _p(w), _p(mu), m, k, B, _COST[ctx.cost], ctx.p,
                                    _p(gout), _p(dX), _p(dU), _p(dY), _p(dmu), _p(ws), nws, C.c_void_p(st)))
        if dmu is not None:
            dmu = dmu.reshape(mu.shape)
        return dU, dY, dX, dmu, None, None, None


def lpcost(U, Y, X, mu, w=None, p=0.25, cost="lp"):
    """Differentiable batched cost; see LpCost."""
    return LpCost.apply(U, Y, X, mu, w, p, cost)
