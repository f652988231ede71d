"""Differentiable H X for PyTorch (adjoint of the matrix-free product).

HApply.apply(X, V, B, op, prec) returns Y = H(V, B) X computed by the HIP
library; its backward, for the cotangent G (PyTorch's convention for complex
tensors, dL = Re sum conj(G) dY), returns
    dL/dX = H G                          (H is Hermitian),
    dL/dV = w|J| Re sum conj(g) x        at the quadrature points,
    dL/dB = w|J| Re sum g^H sigma x      at the quadrature points,
all from chfsi_apply_H_adjoint.  With G = X (M-orthonormal Ritz vectors)
the field gradients are w|J| times the electron and magnetisation densities
of the paper's Sec. II-A: the Hellmann-Feynman gradient of the sum of the
Ritz values (eigsum_grad).
"""
from __future__ import annotations

import torch

from . import binding


class HApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, V, B, op, prec="fp64"):
        op.set_fields(V.detach(), B.detach())
        Y = op.apply_H(X.detach().contiguous(), prec=prec)
        ctx.save_for_backward(X, V, B)
        ctx.op = op
        ctx.prec = prec
        return Y

    @staticmethod
    def backward(ctx, G):
        X, V, B = ctx.saved_tensors
        op = ctx.op
        op.set_fields(V.detach(), B.detach())
        G = G.contiguous().to(X.dtype)
        dX, dV, dB = op.adjoint(X.detach().contiguous(), G, prec=ctx.prec,
                                want_dX=ctx.needs_input_grad[0])
        return dX, dV if ctx.needs_input_grad[1] else None, dB if ctx.needs_input_grad[2] else None, None, None


def happly(X, V, B, op: binding.Chfsi, prec="fp64"):
    return HApply.apply(X, V, B, op, prec)


def eigsum_grad(op: binding.Chfsi, X, prec="fp64"):
    """Gradient of the sum of the Ritz values of the M-orthonormal block X
    with respect to V and B (Hellmann-Feynman): the adjoint with G = X."""
    _, dV, dB = op.adjoint(X, X, prec=prec, want_dX=False)
    return dV, dB
