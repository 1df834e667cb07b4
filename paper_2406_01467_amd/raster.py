"""Plain (one call sequence per batch of views) rasterizer on top of the C ABI,
and the torch.autograd.Function around it.

PyTorch provides device memory and the stream; every step of the path runs in
librade.so's HIP kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import Settings


@dataclasses.dataclass
class ForwardState:
    """Everything rade_render_bwd needs from a forward pass."""
    splats: Optional[torch.Tensor]
    pair_ids: torch.Tensor
    ranges: torch.Tensor
    order: Optional[torch.Tensor]
    t_final: torch.Tensor
    last: torch.Tensor
    median: torch.Tensor
    n_pairs: int
    # the forward's depth and alpha maps (read by the distortion adjoint)
    depth: Optional[torch.Tensor] = None
    alpha: Optional[torch.Tensor] = None
    # the lane masks the forward staged (launch shapes with lane masks only)
    lane_masks: Optional[torch.Tensor] = None


@dataclasses.dataclass
class Maps:
    color: torch.Tensor    # 3 planes per view, packed
    depth: torch.Tensor    # 2 planes per view: expected, median
    normal: torch.Tensor   # 3 planes per view
    alpha: torch.Tensor    # 1 plane per view
    count: Optional[torch.Tensor]
    state: ForwardState
    distortion: Optional[torch.Tensor] = None  # 1 plane per view (Eq. 23), if asked for
    evals: Optional[torch.Tensor] = None       # splats evaluated per pixel, if asked for

    def view_planes(self, rast: "Rasterizer", v: int) -> dict:
        """Per-view (C, H, W) tensors of view v."""
        vw = rast.views_c[v]
        P, o = vw.width * vw.height, vw.pix_offset

        def cut(t, c):
            return t[c * o: c * o + c * P].view(c, vw.height, vw.width)
        out = dict(color=cut(self.color, 3), depth=cut(self.depth, 2), normal=cut(self.normal, 3),
                   alpha=cut(self.alpha, 1), t_final=cut(self.state.t_final, 1),
                   last=cut(self.state.last, 1), median=cut(self.state.median, 1))
        if self.count is not None:
            out["count"] = cut(self.count, 1)
        if self.evals is not None:
            out["evals"] = cut(self.evals, 1)
        if self.distortion is not None:
            out["distortion"] = cut(self.distortion, 1)
        return out


def _aligned16(t: torch.Tensor) -> torch.Tensor:
    t = t.contiguous()
    if t.data_ptr() % 16 != 0:
        t = t.clone()
    return t


class Rasterizer:
    """RaDe-GS rasterizer for a fixed list of views (OpenCV pinhole cameras)."""

    def __init__(self, views: Sequence, settings: Optional[Settings] = None,
                 device="cuda", capacity: int = 0):
        self.settings = settings or Settings()
        self.device = torch.device(device)
        self.views_c = _lib.make_views(views)
        self.total_pixels, self.total_tiles = _lib.rade_views_prepare(self.settings, self.views_c)
        self.views_dev = _lib.views_to_device(self.views_c, self.device)
        self.V = len(views)
        self.capacity = int(capacity)
        self._pairs = None
        self._bin_ws = None
        self._n = -1

    # -- buffers -------------------------------------------------------------
    def _alloc_pairs(self, N: int, capacity: int):
        dev = self.device
        self.capacity = int(capacity)
        self._pairs = torch.empty(max(1, self.capacity), dtype=torch.int32, device=dev)
        ws = _lib.rade_bin_sort_workspace(self.V, N, self.capacity, self.total_tiles)
        self._bin_ws = torch.empty(max(1, ws), dtype=torch.uint8, device=dev)
        self._n = N

    def _new_maps(self, want_count: bool):
        dev, P = self.device, self.total_pixels
        f = lambda c: torch.empty(c * P, dtype=torch.float32, device=dev)  # noqa: E731
        i = lambda: torch.empty(P, dtype=torch.int32, device=dev)  # noqa: E731
        return (f(3), f(2), f(3), f(1), f(1), i(), i(), i() if want_count else None)

    # -- forward -------------------------------------------------------------
    def project(self, means, scales, quats, opacities, sh, stream=None, depth_quad=None):
        """Returns (splats, tiles_touched, bin_records).  depth_quad: (V*N*8,)
        float32 buffer for the exact-depth records (required in
        RADE_DEPTH_EXACT mode)."""
        N = means.shape[0]
        VN = self.V * N
        splats = torch.empty(max(1, VN) * _lib.SPLAT_BYTES, dtype=torch.uint8, device=self.device)
        tt = torch.empty(max(1, VN), dtype=torch.int32, device=self.device)
        brec = torch.empty(4 * max(1, VN), dtype=torch.int32, device=self.device)
        _lib.rade_project(self.settings, self.views_dev, self.V, N, means, scales,
                          _aligned16(quats), opacities, sh, splats, tt, stream, depth_quad, brec)
        return splats, tt, brec

    @property
    def exact_depth(self) -> bool:
        return self.settings.depth_mode == _lib.RADE_DEPTH_EXACT

    def release_pairs(self):
        """Free the pair buffers and binning workspace (reallocated on the
        next bin_sort)."""
        self._pairs = None
        self._bin_ws = None
        self._n = -1

    def bin_sort(self, N: int, tt, brec, want_keys: bool = False, stream=None):
        if self._pairs is None or self._n != N:
            self._alloc_pairs(N, max(self.capacity, 16 * max(N, 1) * self.V // 4 + 1024))
        ranges = torch.empty(2 * max(1, self.total_tiles), dtype=torch.int32, device=self.device)
        n_dev = torch.empty(1, dtype=torch.int64, device=self.device)
        while True:
            keys = (torch.empty(max(1, self.capacity), dtype=torch.int64, device=self.device)
                    if want_keys else None)
            code, M = _lib.rade_bin_sort(self.settings, self.views_c, self.views_dev, self.V, N,
                                         tt, brec, self._pairs, ranges, keys, self.capacity,
                                         n_dev, self._bin_ws, stream, sync_count=True)
            if code == _lib.RADE_OK:
                break
            self._alloc_pairs(N, int(M * 1.25) + 1024)
        pair_ids = self._pairs[:M]
        if want_keys:
            return pair_ids, ranges, M, keys[:M]
        return pair_ids, ranges, M

    def forward(self, means, scales, quats, opacities, sh, want_count: bool = False,
                keep_splats: bool = True, stream=None, want_distortion: bool = False,
                want_evals: bool = False) -> Maps:
        N = means.shape[0]
        quad = (torch.empty(max(1, self.V * N) * 8, dtype=torch.float32, device=self.device)
                if self.exact_depth else None)
        splats, tt, brec = self.project(means, scales, quats, opacities, sh, stream, depth_quad=quad)
        pair_ids, ranges, M = self.bin_sort(N, tt, brec, stream=stream)
        order = self.tile_order(ranges, stream)
        color, depth, normal, alpha, tf, last, med, cnt = self._new_maps(want_count)
        dist = (torch.empty(self.total_pixels, dtype=torch.float32, device=self.device)
                if want_distortion else None)
        evals = (torch.empty(self.total_pixels, dtype=torch.int32, device=self.device)
                 if want_evals else None)
        lm_bytes = _lib.rade_lane_mask_bytes(self.settings, M)
        lane_masks = (torch.empty(max(2, lm_bytes // 8), dtype=torch.int64, device=self.device)
                      if lm_bytes > 0 else None)
        _lib.rade_render_fwd(self.settings, self.views_c, self.views_dev, self.V, N, splats,
                             pair_ids, ranges, color, depth, normal, alpha, tf, last, med, cnt,
                             stream, tile_order=order, distortion=dist, depth_quad=quad,
                             evals=evals, lane_masks=lane_masks)
        # pair_ids are a view of a reusable buffer: keep a private copy for
        # the backward pass
        state = ForwardState(splats if keep_splats else None, pair_ids.clone(), ranges, order,
                             tf, last, med, M, depth, alpha, lane_masks)
        return Maps(color, depth, normal, alpha, cnt, state, dist, evals)

    def tile_order(self, ranges, stream=None):
        """Heavy-first tile order (None for the plain one-workgroup-per-tile
        schedule)."""
        if self.settings.schedule == _lib.RADE_SCHEDULE_TILE:
            return None
        order = torch.empty(self.total_tiles + 1, dtype=torch.int32, device=self.device)
        ws = torch.empty(max(1, _lib.rade_tile_order_workspace(self.total_tiles)),
                         dtype=torch.uint8, device=self.device)
        _lib.rade_tile_order(self.settings, self.views_c, ranges, order, ws, stream)
        return order

    # -- backward ------------------------------------------------------------
    def backward(self, state: ForwardState, means, scales, quats, opacities, sh, d_color=None,
                 d_depth=None, d_normal=None, d_alpha=None, stream=None, d_distortion=None):
        if self.exact_depth:
            raise NotImplementedError("the exact ray-maximum depth (Eq. 7) is a forward-only "
                                      "variant; train with the affine depth of Eq. 4")
        N = means.shape[0]
        recompute = state.splats is None
        ws = _lib.rade_render_bwd_workspace(self.settings, self.V, N, recompute)
        workspace = torch.empty(max(1, ws), dtype=torch.uint8, device=self.device)
        dm = torch.empty_like(means)
        ds = torch.empty_like(scales)
        dq = torch.empty((N, 4), dtype=torch.float32, device=self.device)
        do = torch.empty_like(opacities)
        dsh = torch.empty_like(sh)
        c = lambda t: None if t is None else t.contiguous()  # noqa: E731
        _lib.rade_render_bwd(self.settings, self.views_c, self.views_dev, self.V, N, means, scales,
                             _aligned16(quats), opacities, sh, state.splats, state.pair_ids,
                             state.ranges, state.t_final, state.last, state.median, c(d_color),
                             c(d_depth), c(d_normal), c(d_alpha), dm, ds, dq, do, dsh, workspace,
                             stream, tile_order=state.order, d_distortion=c(d_distortion),
                             depth=state.depth, alpha=state.alpha, lane_masks=state.lane_masks)
        return dm, ds, dq, do, dsh


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rast: Rasterizer, recompute: bool, distortion: bool, means, scales, quats,
                opacities, sh):
        maps = rast.forward(means, scales, quats, opacities, sh, keep_splats=not recompute,
                            want_distortion=distortion)
        ctx.rast = rast
        ctx.state = maps.state
        ctx.distortion = distortion
        ctx.save_for_backward(means, scales, quats, opacities, sh)
        if distortion:
            return maps.color, maps.depth, maps.normal, maps.alpha, maps.distortion
        return maps.color, maps.depth, maps.normal, maps.alpha

    @staticmethod
    def backward(ctx, g_color, g_depth, g_normal, g_alpha, g_dist=None):
        means, scales, quats, opacities, sh = ctx.saved_tensors
        dm, ds, dq, do, dsh = ctx.rast.backward(ctx.state, means, scales, quats, opacities, sh,
                                                g_color, g_depth, g_normal, g_alpha,
                                                d_distortion=g_dist if ctx.distortion else None)
        ctx.state = None
        return None, None, None, dm, ds, dq, do, dsh


def render(rast: Rasterizer, means, scales, quats, opacities, sh, recompute: bool = False,
           distortion: bool = False):
    """Differentiable render of all views of `rast`.  Returns packed planar
    (color [3P], depth [2P], normal [3P], alpha [P]) with P the total pixel
    count, and with distortion=True also the depth-distortion map [P] of
    Eq. 23 (its gradient holds the blend weights constant, as the training
    loss detaches them).  recompute=True keeps no splats for the backward
    pass (they are recomputed from the parameters); the per-pixel blend
    state is always recomputed from the saved final transmittance."""
    return _RenderFn.apply(rast, recompute, distortion, means, scales, quats, opacities, sh)
