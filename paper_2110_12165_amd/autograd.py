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
