"""Differentiable H-matrix product: torch.autograd.Function whose forward is
hmat_matvec and whose backward is hmat_matvec_T (the product kernels run on
the packed blocks of H^T).  H is a constant operator: no gradient flows to
its factors."""
from __future__ import annotations

import torch


class HMatvecFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, H):
        ctx.H = H
        return H.matvec(x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.H.matvec_T(g.contiguous()), None


def hmatvec(H, x):
    """y = H x with gradients d(loss)/dx = H^T d(loss)/dy."""
    return HMatvecFunction.apply(x, H)


class RK45ReplayFunction(torch.autograd.Function):
    """(a, d_c, y_0) -> (y_M, D_M): the rate-and-state integration on a
    frozen list of steps (rs_rk45_replay), differentiated by the discrete
    adjoint (rs_rk45_adjoint) with checkpoints every ckpt_every steps.  b and
    the constants are fixed, so the gradient for a is also the gradient for
    a - b."""

    @staticmethod
    def forward(ctx, a, dc, y0, A, B, b, consts, dts, ckpt_every):
        from . import RK45
        a = a.detach().contiguous()
        dc = dc.detach().contiguous()
        rk = RK45(A, B, a, b.detach().contiguous(), dc, *consts)
        y = y0.detach().clone().contiguous()
        D = torch.zeros(A.n, dtype=torch.float64, device=y.device)
        ctx.ckpt = rk.replay(y, D, dts, ckpt_every=ckpt_every)
        ctx.rk, ctx.dts, ctx.ckpt_every = rk, dts, ckpt_every
        return y, D

    @staticmethod
    def backward(ctx, ybar, Dbar):
        yb = ybar.detach().clone().contiguous()
        _, abar, dcbar = ctx.rk.adjoint(ctx.ckpt, ctx.dts, ctx.ckpt_every, yb, Dbar.detach().contiguous())
        return abar, dcbar, yb, None, None, None, None, None, None


def rk45_replay(A, B, a, b, dc, y0, dts, V0, f0, eta_rad, V_pl, ckpt_every=50):
    """State and slip after the steps dts, differentiable in a, dc and y0.
    A (and B, or None) are HMatrix handles built with transposed products."""
    return RK45ReplayFunction.apply(a, dc, y0, A, B, b, (V0, f0, eta_rad, V_pl), dts, ckpt_every)
