"""torch.autograd.Function over lya_xi / lya_xi_backward.

Forward computes xi(delta, w) with the HIP pair kernel; backward calls the
hand-written HIP backward kernel with dL/dxi.  Positions are not
differentiated (binning is piecewise constant in them) and deltas are taken as
given (no projection inside the graph).
"""
from __future__ import annotations

import torch

from .lya import DeviceForests, Library


class XiFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, delta, weight, lib: Library, forests: DeviceForests, grid, precision: str):
        d = delta.detach().contiguous().to(torch.float64)
        w = weight.detach().contiguous().to(torch.float64)
        out = lib.xi(forests.with_values(delta=d, weight=w), grid, precision=precision)
        ctx.save_for_backward(d, w, out["xi"], out["wsum"])
        ctx.lib, ctx.forests, ctx.grid, ctx.precision = lib, forests, grid, precision
        return out["xi"]

    @staticmethod
    def backward(ctx, grad_xi):
        d, w, xi, wsum = ctx.saved_tensors
        gd, gw = ctx.lib.xi_backward(ctx.forests.with_values(delta=d, weight=w), ctx.grid,
                                     grad_xi.contiguous().to(torch.float64), xi, wsum,
                                     precision=ctx.precision)
        return gd, gw, None, None, None, None


def xi(delta, weight, lib: Library, forests: DeviceForests, grid, precision: str = "fp32"):
    """Differentiable xi [n_realisations, n_bins] as a function of delta and w."""
    return XiFunction.apply(delta, weight, lib, forests, grid, precision)
