"""3D smoothing filter of the Gaussians (the Mip-Splatting filter RaDe-GS
trains with, Sec. 4.1) on top of the C ABI.

`filter3d_var` computes each Gaussian's filter variance from the cameras
(scale / max_view(fx / z)^2 over the views that see its mean); `apply_filter3d`
is a differentiable transform (scales, opacities) -> filtered (scales,
opacities) to feed to the rasterizer, with the variance held constant.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import Settings

FILTER_SCALE = 0.2   # variance of the filter in units of (1 / sampling rate)^2
VIEW_MARGIN = 0.15   # image widened by this fraction on every side for visibility


def filter3d_var(rast, means: torch.Tensor, scale: float = FILTER_SCALE,
                 margin: float = VIEW_MARGIN, settings: Settings | None = None) -> torch.Tensor:
    """Filter variance per Gaussian for the views of `rast` (a Rasterizer)."""
    N = means.shape[0]
    var = torch.empty(N, dtype=torch.float32, device=means.device)
    _lib.rade_filter3d_var(settings or rast.settings, rast.views_dev, rast.V, N,
                           means.contiguous(), scale, margin, var)
    return var


class _Filter3D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scales, opacities, var):
        scales, opacities, var = scales.contiguous(), opacities.contiguous(), var.contiguous()
        N = scales.shape[0]
        s_out = torch.empty_like(scales)
        o_out = torch.empty_like(opacities)
        _lib.rade_filter3d_apply(N, scales, opacities, var, s_out, o_out)
        ctx.save_for_backward(scales, opacities, var)
        return s_out, o_out

    @staticmethod
    def backward(ctx, g_s, g_o):
        scales, opacities, var = ctx.saved_tensors
        N = scales.shape[0]
        g_s = torch.zeros_like(scales) if g_s is None else g_s.contiguous()
        g_o = torch.zeros_like(opacities) if g_o is None else g_o.contiguous()
        d_s = torch.empty_like(scales)
        d_o = torch.empty_like(opacities)
        _lib.rade_filter3d_apply_bwd(N, scales, opacities, var, g_s, g_o, d_s, d_o)
        return d_s, d_o, None


def apply_filter3d(scales: torch.Tensor, opacities: torch.Tensor, var: torch.Tensor):
    """Filtered (scales, opacities): sqrt(s^2 + var) per axis and
    o * sqrt(prod s^2 / prod (s^2 + var)); differentiable in scales and
    opacities (var is a constant)."""
    return _Filter3D.apply(scales, opacities, var)
