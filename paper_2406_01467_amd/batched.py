"""Batched multi-view rendering: one launch per kernel over many views of
uneven size, the whole forward + backward captured in a HIP graph, and an
autotuner for the tile size, the work schedule, the wave shape and the staging
batch.

All views share one key space (global tile = view's tile offset + tile), so
each kernel of the path is launched once for the whole batch; the render
kernels can visit tiles longest-list first, either one workgroup per tile or
with resident workgroups pulling tiles from a device counter.  A plan
allocates every buffer up front; its step enqueues project -> bin/sort (no
host synchronisation: the pair count stays on the device) -> tile order ->
render forward -> upstream gradients (caller's elementwise function) ->
render backward -> projection backward.  After a replay, `overflowed()`
reads the device pair count once; on overflow the plan grows its capacity
and captures again.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Callable, Optional, Sequence

import torch

from . import _lib
from ._lib import Settings
from .raster import Rasterizer


class BatchedPlan:
    """Pre-allocated fwd+bwd of N Gaussians over a fixed list of views.

    params: the five parameter tensors (means, scales, quats, opacities, sh);
    the plan keeps references (their storage must stay put; update in place).
    grad_fn(maps) -> (d_color, d_depth, d_normal, d_alpha) computes upstream
    gradients from the map tensors with stream-ordered torch ops; under graph
    capture it must avoid host synchronisation (elementwise ops are safe).
    With distortion=True the forward also writes maps["distortion"] (Eq. 23)
    and grad_fn returns a fifth gradient, that of the distortion map.
    """

    def __init__(self, views: Sequence, settings: Settings, params: Sequence[torch.Tensor],
                 grad_fn: Callable, capacity: Optional[int] = None, recompute: bool = False,
                 distortion: bool = False):
        if settings.depth_mode != _lib.RADE_DEPTH_AFFINE:
            raise ValueError("a training step needs the affine depth of Eq. 4 (the exact "
                             "ray-maximum depth is a forward-only variant)")
        self.settings = settings
        self.params = [p.detach() for p in params]
        self.device = self.params[0].device
        self.N = self.params[0].shape[0]
        self.rast = Rasterizer(views, settings, self.device)
        self.V = self.rast.V
        self.grad_fn = grad_fn
        self.recompute = recompute
        self.distortion = distortion
        self.graph = None
        if capacity is None:
            # one eager binning pass sizes the pair buffers (with slack); the
            # rasterizer's buffers for it are released after
            splats, tt, brec = self.rast.project(*self.params)
            _, _, M = self.rast.bin_sort(self.N, tt, brec)
            del splats, tt, brec
            self.rast.release_pairs()
            capacity = int(M * 1.15) + 4096
        self._alloc(capacity)

    # -- buffers -------------------------------------------------------------
    def _alloc(self, capacity: int):
        dev, V, N, r = self.device, self.V, self.N, self.rast
        VN = max(1, V * N)
        self.capacity = int(capacity)
        self.pair_ids = torch.empty(max(1, self.capacity), dtype=torch.int32, device=dev)
        self.ranges = torch.empty(2 * max(1, r.total_tiles), dtype=torch.int32, device=dev)
        self.n_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        # One arena holds the binning workspace and the backward's workspace.
        # The binning workspace is scratch of rade_bin_sort only, and the
        # backward's gradient records (its first V x N x 64 bytes) are
        # written after its start and read by its end: stream order keeps the
        # two apart, so they share memory.  With recompute, the backward
        # recomputes the splat records and tile counts into its workspace
        # after the gradient records (rade.h gives the layout); the forward
        # projects into that same region, so no second copy of the V x N
        # records exists, and the region lies after the binning workspace,
        # which reads the records while it runs.  The 16-byte binning records
        # are read by rade_bin_sort while its workspace is in use: they lie
        # beyond it (after the backward's regions with recompute, else
        # between the binning workspace and the arena's end).
        a256 = lambda b: (b + 255) & ~255  # noqa: E731
        bin_bytes = a256(max(1, _lib.rade_bin_sort_workspace(V, N, self.capacity,
                                                             r.total_tiles)))
        bwd_bytes = a256(max(1, _lib.rade_render_bwd_workspace(self.settings, V, N,
                                                               self.recompute)))
        g_bytes = a256(V * N * 16 * 4)
        brec_bytes = a256(16 * VN)
        if self.recompute and V * N > 0:
            head = max(bin_bytes, g_bytes)
            end = head - g_bytes + bwd_bytes
            self.arena = torch.empty(end + brec_bytes, dtype=torch.uint8, device=dev)
            self.bwd_ws = self.arena[head - g_bytes: end]
            self.brec = self.arena[end: end + 16 * VN].view(torch.int32)
            s_bytes = V * N * _lib.SPLAT_BYTES
            self.splats = self.arena[head: head + s_bytes]
            t0 = head + a256(s_bytes)
            self.tt = self.arena[t0: t0 + 4 * V * N].view(torch.int32)
        else:
            self.arena = torch.empty(max(bin_bytes + brec_bytes, bwd_bytes), dtype=torch.uint8,
                                     device=dev)
            self.bwd_ws = self.arena[:bwd_bytes]
            self.brec = self.arena[bin_bytes: bin_bytes + 16 * VN].view(torch.int32)
            self.splats = torch.empty(VN * _lib.SPLAT_BYTES, dtype=torch.uint8, device=dev)
            self.tt = torch.empty(VN, dtype=torch.int32, device=dev)
        self.bin_ws = self.arena[:bin_bytes]
        # the lane masks the forward stages, read back by the backward (launch
        # shapes with lane masks only; written and read while the gradient
        # records are live, so not in the arena)
        lm_bytes = _lib.rade_lane_mask_bytes(self.settings, self.capacity)
        self.lane_masks = (torch.empty(max(2, lm_bytes // 8), dtype=torch.int64, device=dev)
                           if lm_bytes > 0 else None)
        self.order = torch.empty(r.total_tiles + 1, dtype=torch.int32, device=dev)
        self.order_ws = torch.empty(max(1, _lib.rade_tile_order_workspace(r.total_tiles)),
                                    dtype=torch.uint8, device=dev)
        P = r.total_pixels
        f = lambda c: torch.zeros(c * P, dtype=torch.float32, device=dev)  # noqa: E731
        i = lambda: torch.zeros(P, dtype=torch.int32, device=dev)  # noqa: E731
        self.maps = dict(color=f(3), depth=f(2), normal=f(3), alpha=f(1), t_final=f(1),
                         last=i(), median=i())
        if self.distortion:
            self.maps["distortion"] = f(1)
        m, s, q, o, sh = self.params
        self.grads = [torch.zeros_like(m), torch.zeros_like(s), torch.zeros((N, 4), device=dev),
                      torch.zeros_like(o), torch.zeros_like(sh)]
        self.graph = None

    # -- the step --------------------------------------------------------------
    def enqueue(self):
        """Enqueue one fwd+bwd on the current stream (no host sync)."""
        st, r, V, N = self.settings, self.rast, self.V, self.N
        m, s, q, o, sh = self.params
        _lib.rade_project(st, r.views_dev, V, N, m, s, q, o, sh, self.splats, self.tt,
                          bin_records=self.brec)
        _lib.rade_bin_sort(st, r.views_c, r.views_dev, V, N, self.tt, self.brec, self.pair_ids,
                           self.ranges, None, self.capacity, self.n_dev, self.bin_ws,
                           sync_count=False)
        order = None
        if st.schedule != _lib.RADE_SCHEDULE_TILE:
            _lib.rade_tile_order(st, r.views_c, self.ranges, self.order, self.order_ws)
            order = self.order
        mp = self.maps
        _lib.rade_render_fwd(st, r.views_c, r.views_dev, V, N, self.splats, self.pair_ids,
                             self.ranges, mp["color"], mp["depth"], mp["normal"], mp["alpha"],
                             mp["t_final"], mp["last"], mp["median"], None, tile_order=order,
                             distortion=mp.get("distortion"), lane_masks=self.lane_masks)
        g = self.grad_fn(mp)
        g = [None if x is None else x.contiguous() for x in g]
        dc, dd, dn, da = g[:4]
        ddist = g[4] if self.distortion and len(g) > 4 else None
        _lib.rade_render_bwd(st, r.views_c, r.views_dev, V, N, m, s, q, o, sh,
                             None if self.recompute else self.splats, self.pair_ids, self.ranges,
                             mp["t_final"], mp["last"], mp["median"], dc, dd, dn, da,
                             *self.grads, self.bwd_ws, tile_order=order, d_distortion=ddist,
                             depth=mp["depth"], alpha=mp["alpha"], lane_masks=self.lane_masks)

    def capture(self):
        """Capture enqueue() into a HIP graph (after one eager warm-up)."""
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.enqueue()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.enqueue()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def n_pairs(self) -> int:
        return int(self.n_dev.item())

    def overflowed(self) -> bool:
        return self.n_pairs() > self.capacity

    def step(self, check: bool = True) -> int:
        """Replay once; when check, verify the pair count and, on overflow,
        grow, re-capture and replay.  Returns the number of replays made."""
        self.replay()
        if not check or not self.overflowed():
            return 1
        self._alloc(int(self.n_pairs() * 1.25) + 4096)
        self.capture()
        self.replay()
        return 2


# ---------------------------------------------------------------------------
# Autotuner

TILES = [(8, 8), (16, 16), (16, 32), (32, 16)]
SCHEDULES = [_lib.RADE_SCHEDULE_TILE, _lib.RADE_SCHEDULE_HEAVY_FIRST, _lib.RADE_SCHEDULE_PERSISTENT]


def _cache_path() -> str:
    base = os.environ.get("RADE_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rade", "autotune.json"))
    return base


def signature(views: Sequence, n: int, sh_degree: int) -> str:
    h = hashlib.sha1()
    h.update(f"{n}:{sh_degree}:".encode())
    for v in views:
        h.update(f"{v.width}x{v.height};".encode())
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{dev}|{h.hexdigest()[:16]}"


WAVE_WIDTHS = (8, 16, 32)   # 8x8, 16x4, 32x2 pixels per wavefront
BATCHES = (0, 64, 128, 256)  # splats staged per round (0: one per thread)


def _shape_fits(tw: int, th: int, ww: int) -> bool:
    return tw % ww == 0 and th % (64 // ww) == 0


def autotune(views: Sequence, params: Sequence[torch.Tensor], base: Settings, grad_fn: Callable,
             tiles=TILES, schedules=SCHEDULES, wave_widths=WAVE_WIDTHS, batches=BATCHES,
             reps: int = 3, use_cache: bool = True, log: Optional[Callable] = None,
             distortion: bool = False) -> tuple:
    """Time the graph-replayed fwd+bwd over the candidates and return (best
    Settings, {candidate: ms}).  Two stages: every (tile, schedule), with and
    without lane masks on tiles of several 8x8 waves, then, for the best
    plain shape of those, every wave shape the tile holds x staging batch
    (the tuned shapes exist for the plain path only, so not with the
    distortion term).  Results are cached in a JSON file keyed by device
    name and workload signature."""
    sig = signature(views, params[0].shape[0], base.sh_degree) + ("|dist" if distortion else "")
    sig += "|shape|lm"
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and sig in cache:
        c = cache[sig]
        return Settings(**{**base.__dict__, "tile_w": c["tile_w"], "tile_h": c["tile_h"],
                           "schedule": c["schedule"], "wave_w": c.get("wave_w", 0),
                           "batch": c.get("batch", 0),
                           "lane_masks": c.get("lane_masks", 0)}), c.get("timings", {})
    timings = {}

    def timed(st: Settings, key: str) -> float:
        plan = BatchedPlan(views, st, params, grad_fn, distortion=distortion)
        plan.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.replay()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        del plan
        timings[key] = ms
        if log:
            log(f"autotune {key}: {ms:.3f} ms")
        return ms

    best = None
    best_plain = None
    for tw, th in tiles:
        for sch in schedules:
            st = Settings(**{**base.__dict__, "tile_w": tw, "tile_h": th, "schedule": sch,
                             "wave_w": 0, "batch": 0, "lane_masks": 0})
            ms = timed(st, f"{tw}x{th}/{sch}")
            if best is None or ms < best[0]:
                best = (ms, st)
            if best_plain is None or ms < best_plain[0]:
                best_plain = (ms, st)
            if not distortion and tw * th > 64:
                st = Settings(**{**st.__dict__, "lane_masks": 1})
                ms = timed(st, f"{tw}x{th}/{sch}/lm")
                if ms < best[0]:
                    best = (ms, st)
    if not distortion:
        b = best_plain[1]
        for ww in wave_widths:
            if not _shape_fits(b.tile_w, b.tile_h, ww):
                continue
            for bt in batches:
                if (ww == 8 and bt in (0, b.tile_w * b.tile_h)):
                    continue  # the default shape, timed in the first stage
                st = Settings(**{**b.__dict__, "wave_w": ww, "batch": bt})
                ms = timed(st, f"{b.tile_w}x{b.tile_h}/{b.schedule}/w{ww}/b{bt}")
                if ms < best[0]:
                    best = (ms, st)
    if use_cache:
        cache[sig] = dict(tile_w=best[1].tile_w, tile_h=best[1].tile_h,
                          schedule=best[1].schedule, wave_w=best[1].wave_w,
                          batch=best[1].batch, lane_masks=best[1].lane_masks, timings=timings)
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best[1], timings
