"""The training loss used to exercise the rasterizer: L1 on colour plus
w_n x the normal-consistency term of Sec. 3.4, Eq. 24 (w_n = 5, Sec. 4.1),
with the normal n~ taken from the median-depth map by central differences of
back-projected points and not detached; optionally plus w_d x the mean over
pixels of the depth distortion of Eq. 23 (w_d = 100 in Sec. 4.1; its
gradient holds the blend weights constant).

`make_grad_fn` returns the upstream gradients into pre-allocated buffers
(the library's kernels for the L1 term and for Eq. 24, both writing their
maps whole, so nothing is cleared first), safe under HIP-graph capture;
`torch_loss` is the same loss in torch ops for the autograd path.
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

from . import _lib

W_NORMAL = 5.0
W_DIST = 100.0


def make_grad_fn(rast, target, w_normal: float = W_NORMAL, w_dist: float = 0.0):
    """Upstream gradients of the benchmark loss into pre-allocated buffers:
    L1 colour (library kernel, mean per view) + w_normal x Eq. 24 (fused
    library kernel, overwriting the depth, normal and alpha gradient maps)
    [+ w_dist x mean distortion (Eq. 23): a constant gradient map, returned
    fifth].  Safe inside a HIP graph: no allocation, no host sync."""
    dev, P = rast.device, rast.total_pixels
    target = target.contiguous()
    dC = torch.empty(3 * P, dtype=torch.float32, device=dev)
    dDNA = torch.empty(6 * P, dtype=torch.float32, device=dev)
    dD, dN, dA = dDNA[:2 * P], dDNA[2 * P:5 * P], dDNA[5 * P:]
    loss = torch.empty(rast.V, dtype=torch.float32, device=dev)
    dL = None
    if w_dist > 0.0:
        dL = torch.empty(P, dtype=torch.float32, device=dev)
        for vc in rast.views_c:
            n = vc.width * vc.height
            dL[vc.pix_offset: vc.pix_offset + n] = w_dist / n
    ws = torch.empty(max(1, _lib.rade_normal_consistency_workspace(P)), dtype=torch.uint8,
                     device=dev)

    def grad_fn(maps):
        _lib.rade_l1_color_grad(rast.views_c, rast.views_dev, maps["color"], target, 1.0, dC)
        _lib.rade_normal_consistency(rast.views_c, rast.views_dev, maps["depth"], maps["normal"],
                                     maps["alpha"], w_normal, loss, dD, dN, dA, ws,
                                     accumulate=False)
        if dL is not None:
            return dC, dD, dN, dA, dL
        return dC, dD, dN, dA

    grad_fn.loss = loss
    return grad_fn


def torch_loss(color, depth, normal, alpha, target, views_c, w_normal: float = W_NORMAL,
               distortion=None, w_dist: float = 0.0):
    """The same loss written with torch ops (eager autograd path)."""
    total = color.new_zeros(())
    for vc in views_c:
        H, W, o = vc.height, vc.width, vc.pix_offset
        P = H * W
        C = color[3 * o: 3 * o + 3 * P].view(3, H, W)
        D = depth[2 * o: 2 * o + 2 * P].view(2, H, W)[1]
        Nm = normal[3 * o: 3 * o + 3 * P].view(3, H, W)
        A = alpha[o: o + P].view(H, W)
        T = target[3 * o: 3 * o + 3 * P].view(3, H, W)
        u = (torch.arange(W, device=C.device, dtype=C.dtype) + 0.5 - vc.cx) / vc.fx
        v = (torch.arange(H, device=C.device, dtype=C.dtype) + 0.5 - vc.cy) / vc.fy
        X = torch.stack([D * u[None, :], D * v[:, None], D], 0)
        du = X[:, 1:-1, 2:] - X[:, 1:-1, :-2]
        dv = X[:, 2:, 1:-1] - X[:, :-2, 1:-1]
        n = F.normalize(torch.cross(du, dv, dim=0), dim=0)
        facing = torch.where((n * X[:, 1:-1, 1:-1]).sum(0) > 0, -1.0, 1.0)
        l_n = (A[1:-1, 1:-1] - (Nm[:, 1:-1, 1:-1] * n * facing).sum(0)).mean()
        total = total + (C - T).abs().mean() + w_normal * l_n
        if distortion is not None and w_dist > 0.0:
            total = total + w_dist * distortion[o: o + P].mean()
    return total
