"""torch.autograd.Function wrappers of the PD / FD equalisers.

Forward and backward both run in libdbpeq.so (the backward is the library's
hand-written adjoint, not autograd tracing).  N0 is a 0-dim tensor whose value
is passed to the library as a host float; its gradient comes back as a
0-dim tensor on N0's device.  Complex gradients follow PyTorch's convention
(dL/dRe + i dL/dIm).
"""
from __future__ import annotations

import torch

from . import api


def _n0_value(n0) -> float:
    return float(n0.detach().cpu()) if isinstance(n0, torch.Tensor) else float(n0)


class EqPD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H, y, n0, cluster_off, es=1.0):
        n0v = _n0_value(n0)
        z, s2 = api.eq_pd(H.detach(), y.detach(), n0v, cluster_off, precision="fp32", es=es)
        ctx.save_for_backward(H.detach(), y.detach())
        ctx.n0v, ctx.off, ctx.es = n0v, cluster_off, es
        ctx.n0_like = n0 if isinstance(n0, torch.Tensor) else None
        return z, s2

    @staticmethod
    def backward(ctx, gz, gs):
        H, y = ctx.saved_tensors
        gH, gy, gn0 = api.eq_pd_backward(H, y, ctx.n0v, ctx.off, gz=gz, gs=gs, es=ctx.es)
        g_n0 = None
        if ctx.n0_like is not None and ctx.needs_input_grad[2]:
            g_n0 = gn0.to(device=ctx.n0_like.device, dtype=ctx.n0_like.dtype)
        return (gH if ctx.needs_input_grad[0] else None, gy if ctx.needs_input_grad[1] else None,
                g_n0, None, None)


class EqFD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H, y, n0, cluster_off, nu=None, es=1.0):
        n0v = _n0_value(n0)
        nud = None if nu is None else nu.detach()
        z, s2 = api.eq_fd(H.detach(), y.detach(), n0v, cluster_off, nu=nud, precision="fp32", es=es)
        ctx.save_for_backward(H.detach(), y.detach(), nud if nud is not None else torch.empty(0))
        ctx.has_nu = nu is not None
        ctx.n0v, ctx.off, ctx.es = n0v, cluster_off, es
        ctx.n0_like = n0 if isinstance(n0, torch.Tensor) else None
        return z, s2

    @staticmethod
    def backward(ctx, gz, gs):
        H, y, nu = ctx.saved_tensors
        gH, gy, gn0, gnu = api.eq_fd_backward(H, y, ctx.n0v, ctx.off, gz=gz, gs=gs,
                                              nu=nu if ctx.has_nu else None, es=ctx.es)
        g_n0 = None
        if ctx.n0_like is not None and ctx.needs_input_grad[2]:
            g_n0 = gn0.to(device=ctx.n0_like.device, dtype=ctx.n0_like.dtype)
        return (gH if ctx.needs_input_grad[0] else None, gy if ctx.needs_input_grad[1] else None,
                g_n0, None, gnu if (ctx.has_nu and ctx.needs_input_grad[4]) else None, None)


def eq_pd(H, y, n0, cluster_off, es=1.0):
    """Differentiable PD L-MMSE: (z, sigma2)."""
    return EqPD.apply(H, y, n0, cluster_off, es)


def eq_fd(H, y, n0, cluster_off, nu=None, es=1.0):
    """Differentiable FD L-MMSE: (z, sigma2); nu (optional) receives a gradient."""
    return EqFD.apply(H, y, n0, cluster_off, nu, es)
