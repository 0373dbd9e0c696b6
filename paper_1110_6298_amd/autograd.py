"""Reverse-mode differentiation of the MW transforms for PyTorch.

``MWForward`` and ``MWInverse`` are ``torch.autograd.Function``s whose backward
passes call the library's adjoint entry points: for a linear map y = A x and a
real loss, PyTorch's complex gradient convention (d/dRe + i d/dIm) gives
grad_x = A^H grad_y, and for real maps (reality = 1) the real part of it.

Inputs may carry one leading batch dimension; a batch runs as one library call.
"""
from __future__ import annotations

import torch

from . import FP64, _batch

__all__ = ["MWForward", "MWInverse", "forward", "inverse"]


def _split(x, lead):
    """Views of the maps of a batched tensor (or the tensor itself)."""
    return [x[b] for b in range(x.shape[0])] if lead else [x]


def _apply(name, x, L, spin, reality, precision, lead):
    xs = _split(x.contiguous(), lead)
    n = len(xs)
    outs = _batch(name, xs, [L] * n, [spin] * n, [reality] * n, precision, None, None)
    return torch.stack(outs) if lead else outs[0]


class MWForward(torch.autograd.Function):
    """coefficients = forward(map); backward: grad_map = forward_adjoint(grad_coeffs)."""

    @staticmethod
    def forward(ctx, x, L, spin=0, reality=0, precision=FP64):
        lead = x.dim() == 3
        ctx.args = (L, spin, reality, precision, lead)
        return _apply("mw_forward", x, L, spin, reality, precision, lead)

    @staticmethod
    def backward(ctx, g):
        L, spin, reality, precision, lead = ctx.args
        gx = _apply("mw_forward_adjoint", g.to(torch.complex128), L, spin, reality, precision, lead)
        return gx, None, None, None, None


class MWInverse(torch.autograd.Function):
    """map = inverse(coefficients); backward: grad_coeffs = inverse_adjoint(grad_map)."""

    @staticmethod
    def forward(ctx, flm, L, spin=0, reality=0, precision=FP64):
        lead = flm.dim() == 2
        ctx.args = (L, spin, reality, precision, lead)
        return _apply("mw_inverse", flm, L, spin, reality, precision, lead)

    @staticmethod
    def backward(ctx, g):
        L, spin, reality, precision, lead = ctx.args
        dt = torch.float64 if reality else torch.complex128
        gc = _apply("mw_inverse_adjoint", g.to(dt), L, spin, reality, precision, lead)
        return gc, None, None, None, None


def forward(x, L: int, spin: int = 0, reality: int = 0, precision=FP64):
    """Differentiable forward transform of a map (L, 2L-1) or a batch (B, L, 2L-1)."""
    return MWForward.apply(x, L, spin, reality, precision)


def inverse(flm, L: int, spin: int = 0, reality: int = 0, precision=FP64):
    """Differentiable inverse transform of (L*L,) or (B, L*L) coefficients."""
    return MWInverse.apply(flm, L, spin, reality, precision)
