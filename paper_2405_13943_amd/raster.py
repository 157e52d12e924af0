"""Differentiable rasterization as a ``torch.autograd.Function``.

Forward = ``gs_project`` -> ``gs_bin_sort`` -> ``gs_render_fwd``; backward =
``gs_render_bwd`` fed the incoming dL/dC (external-gradient mode).  The
transmittance is recomputed in the backward, never stored per pair; the
saved state is the projected records, the tile bins and the rendered image.

FP32 and FP64 parameter planes are both accepted (the FP64 path runs the
same kernels instantiated for double and serves the adjoint checks).
"""
from __future__ import annotations

import torch

from . import gs


class GaussianRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, frame: gs.Frame, cfg: gs.GsRasterCfg, capacity=None):
        """params: [A][N] planes on the GPU.  Returns the frame's colour
        buffer (all jobs' [3][H][W] images back to back)."""
        buf = gs.rasterize(params.detach(), frame, cfg, capacity=capacity)
        ctx.frame, ctx.cfg, ctx.buf = frame, cfg, buf
        ctx.save_for_backward(params)
        return buf.rgb.clone()

    @staticmethod
    def backward(ctx, grad_rgb: torch.Tensor):
        (params,) = ctx.saved_tensors
        grad = torch.empty_like(params)
        gs.render_bwd(params.detach(), ctx.frame, ctx.cfg, ctx.buf, grad, gs.LOSS_EXTERNAL,
                      grad_rgb.contiguous())
        return grad, None, None, None


def rasterize(params: torch.Tensor, frame: gs.Frame, cfg: gs.GsRasterCfg, capacity=None) -> torch.Tensor:
    return GaussianRasterize.apply(params, frame, cfg, capacity)
