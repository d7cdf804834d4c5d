"""torch.autograd.Function over lya_xi / lya_xi_backward.

Forward computes xi(delta, w) with the HIP pair kernel; backward calls the
hand-written HIP backward kernel with dL/dxi.  Positions are not
differentiated (binning is piecewise constant in them).  With
``project_deltas`` the forward correlates eta delta per forest (Sec. 2.2) and
the gradients are those of the raw delta and w, through eta's dependence on w.
"""
from __future__ import annotations

import torch

from .lya import DeviceForests, Library


class XiFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, delta, weight, lib: Library, forests: DeviceForests, grid, precision: str,
                project_deltas: bool, eta: str):
        d = delta.detach().contiguous().to(torch.float64)
        w = weight.detach().contiguous().to(torch.float64)
        ctx.opts = dict(precision=precision, project_deltas=project_deltas, eta=eta)
        out = lib.xi(forests.with_values(delta=d, weight=w), grid, **ctx.opts)
        ctx.save_for_backward(d, w, out["xi"], out["wsum"])
        ctx.lib, ctx.forests, ctx.grid = lib, forests, grid
        return out["xi"]

    @staticmethod
    def backward(ctx, grad_xi):
        d, w, xi, wsum = ctx.saved_tensors
        gd, gw = ctx.lib.xi_backward(ctx.forests.with_values(delta=d, weight=w), ctx.grid,
                                     grad_xi.contiguous().to(torch.float64), xi, wsum, **ctx.opts)
        return gd, gw, None, None, None, None, None, None


def xi(delta, weight, lib: Library, forests: DeviceForests, grid, precision: str = "fp32",
       project_deltas: bool = False, eta: str = "mean_slope"):
    """Differentiable xi [n_realisations, n_bins] as a function of delta and w
    (of the projected deltas' xi when ``project_deltas``)."""
    return XiFunction.apply(delta, weight, lib, forests, grid, precision, project_deltas, eta)
