#!/usr/bin/env python3
"""Benchmark of the RaDe-GS rasterizer hot path on one MI355X.

One step = one forward + backward pass of the whole path over every view of
the workload: projection with SH (FP64 geometry), binning and the depth/tile
radix sorts, the tile rasterizer forward (colour, expected and median depth,
normal, alpha), the loss gradient, the rasterizer backward and the
projection backward.  The loss is L1(colour, target) + 5 x the
normal-consistency term of Eq. 24 (alpha - N . n~ over interior pixels, n~
from the median-depth map, not detached; w_n = 5 as in Sec. 4.1); its
gradient is computed by torch elementwise ops (L1) and the library's fused
kernel (Eq. 24).  The whole step is captured once in a HIP graph and
replayed; the pair count stays on the device and is checked after the timed
replays.  Inputs are seeded synthetic and resident in HBM before timing.

Default workload: 1,000,000 Gaussians (64 anisotropic clusters at distance
2..20, SH degree 3) seen by one 1600x1064 view.

Prints one JSON line: value = splat-pixel blends per second, ms_per_step =
fwd+bwd milliseconds per step (all views), ms_per_view = the same per view;
the roofline of the dominant kernel (its duration from HIP events the library
records around its launches; algorithmic flops against the FP32 vector peak
and algorithmic bytes against the HBM peak) and of the whole step; the
evaluations per blend (splats the pixels evaluated over splats they blended);
the eager autograd path (torch.autograd.Function + torch loss) for
comparison; the many-view leg: 16 uneven views of the same scene rendered as
one batch, against the same views unbatched; the FP64 CPU oracle timed on a
bounded pixel sample.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ms/view and splat-pixel blends/s, 1M Gaussians, 1600x1064"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak (packed FP32 instructions)
# The FP32 vector peak without packed instructions (this library emits none):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6
PEAK_HBM_GBS = 8000.0         # MI355X published HBM3E bandwidth

# Algorithmic FP32 operations per blended (pixel, splat) pair, counted from
# the method's arithmetic (FMA = 2): forward = offset (2), quadratic form (8),
# exp (1), alpha (1), 1-alpha and T (2), weight (1), colour (6), depth plane
# (4) and its blend (2), normal (6), alpha sum (1) = 34; backward = the same
# alpha (14), T recovery (2), weight (1), depth plane (4), upstream dot
# product (17), d alpha (4), running sum (2), depth grad (3), d power (2),
# centre grads (8), conic grads (7), opacity (1), colour (3), depth/plane (3),
# normal (3) = 74.
FLOPS_PER_BLEND = {"render_fwd": 34, "render_bwd": 74}

# Algorithmic HBM bytes of one fwd+bwd step: the least traffic the method
# moves, ignoring multiple radix passes and atomics.
#  - per Gaussian, once per batch of views: parameters read, read again by the
#    backward, parameter gradients written: 3 x 4 (11 + 3K) bytes (708 at SH
#    degree 3, K = 16);
#  - per (Gaussian, view): splat record written 68, tile count written and
#    scanned 8, support rect read 16, splat-gradient record written and read
#    60 + 60 = 212;
#  - per (tile, splat) pair: emitted 12, sorted 24, ranges 8, gathered by the
#    forward 68 and by the backward 68 = 180;
#  - per pixel: maps and saved state written by the forward 48, read by the
#    backward 48 = 96.
# The rasterizer backward alone moves 68 per pair (gather), 48 per pixel
# (upstream gradients and saved state) and 60 per (Gaussian, view) (its
# gradient-record writes).
def param_bytes(sh_degree: int) -> int:
    return 4 * (11 + 3 * (sh_degree + 1) ** 2)


BYTES_PER_GAUSSIAN_VIEW = 68 + 8 + 16 + 60 + 60
BYTES_PER_PAIR = 12 + 24 + 8 + 68 + 68
BYTES_PER_PIXEL = 48 + 48
RENDER_BWD_BYTES = {"pair": 68, "pixel": 48, "gaussian_view": 60}
RENDER_FWD_BYTES = {"pair": 68, "pixel": 48, "gaussian_view": 0}


def step_bytes(n: int, views: int, pairs: int, pixels: int, sh_degree: int) -> int:
    return (3 * param_bytes(sh_degree) * n + BYTES_PER_GAUSSIAN_VIEW * n * views +
            BYTES_PER_PAIR * pairs + BYTES_PER_PIXEL * pixels)


def kernel_bytes(kernel: str, n: int, views: int, pairs: int, pixels: int) -> int:
    c = RENDER_BWD_BYTES if kernel == "render_bwd" else RENDER_FWD_BYTES
    return c["pair"] * pairs + c["pixel"] * pixels + c["gaussian_view"] * n * views


# HBM traffic of one launch of the dominant kernel, from two rocprofv3 --pmc
# runs of paper_2406_01467_amd/profile_step.py (FETCH_SIZE, then WRITE_SIZE,
# KiB per dispatch), each scaled by what the counter reads for a copy kernel
# of known size (FETCH_SIZE reads half of the bytes a plain copy moves,
# WRITE_SIZE all of them), and its VALU counters from a third run (VALU
# issue = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x duration x 2.4 GHz)).
# Valid only for the kernel sources they were measured on (SHA-1 of
# render.hip + common.hpp) and for the workload in the launch configuration
# they were measured in (tile, schedule, wave shape, batch, lane masks); reported as null
# otherwise.
MEASURED = [
    {"kernel": "render_bwd", "workload": "plain_1600x1064_1m", "tile": "16x16",
     "schedule": 1, "wave_w": 0, "batch": 0, "lane_masks": 0,
     "sources_sha1": "208baf9f505f40f3b6b7fac587f2e696860e6b1a",
     "fetch_bytes": 374570923, "write_bytes": 154785088, "valu_issue": 0.83,
     "profile": "profiles/kernels_1600x1064_1m_pmc.md"},
    {"kernel": "render_bwd", "workload": "batched_16views_1m", "tile": "16x16",
     "schedule": 1, "wave_w": 0, "batch": 0, "lane_masks": 1,
     "sources_sha1": "208baf9f505f40f3b6b7fac587f2e696860e6b1a",
     "fetch_bytes": 6221583181, "write_bytes": 2709135936, "valu_issue": 0.86,
     "profile": "profiles/kernels_batched_16views_1m_pmc.md"},
]


# Launch settings of the 16-view batch, as the autotuner chose them over tile
# size x schedule x lane masks, then wave shape x staging batch (`--tile auto`
# with `--workload batched_16views_1m`); fixed here so the timed run does no
# tuning.
BATCHED_TUNED = {"tile": "16x16", "schedule": 1, "batch": 0, "wave_w": 0, "lane_masks": 1}


def _render_sources_sha1() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in ("render.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2406_01467_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured(kernel: str, workload: str, settings, distortion: bool = False):
    if distortion:  # the counters were taken on the kernels without Eq. 23
        return None
    tile = f"{settings.tile_w}x{settings.tile_h}"
    sha = _render_sources_sha1()
    for t in MEASURED:
        if (t["kernel"] == kernel and t["workload"] == workload and t["tile"] == tile
                and t["schedule"] == settings.schedule and t["wave_w"] == settings.wave_w
                and t["batch"] == settings.batch
                and t.get("lane_masks", 0) == settings.lane_masks and t["sources_sha1"] == sha):
            return t
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="plain_1600x1064_1m")
    ap.add_argument("--tile", default="16x16", help="WxH, or 'auto' (autotune)")
    ap.add_argument("--schedule", type=int, default=1,
                    help="0: one workgroup per tile, 1: heavy first (default, the autotuner's choice "
                         "for the default workload), 2: persistent")
    ap.add_argument("--lane-masks", type=int, default=0,
                    help="1: lane masks on every 8x8 wave of larger tiles (rade_settings.lane_masks)")
    ap.add_argument("--cpu-pixels", type=int, default=4096,
                    help="pixels of the oracle's CPU-baseline sample (0: skip)")
    ap.add_argument("--eager-steps", type=int, default=5,
                    help="steps of the eager autograd path timed for comparison (0: skip)")
    ap.add_argument("--recompute", action="store_true",
                    help="keep no splats for the backward pass")
    ap.add_argument("--distortion", action="store_true",
                    help="add w_d = 100 x the depth distortion of Eq. 23 to the loss")
    ap.add_argument("--depth-ablation", type=int, default=0, metavar="K",
                    help="also time K forward passes with the affine depth (Eq. 4) and with "
                         "the exact ray-maximum depth (Eq. 7) and compare the depth maps")
    ap.add_argument("--mesh-grid", type=int, default=0, metavar="R",
                    help="also fuse the views' median depth into an R^3 TSDF grid and mesh it "
                         "with Marching Cubes (mesh extraction, Sec. 4.1), timed")
    ap.add_argument("--unbatched-steps", type=int, default=5,
                    help="with several views: steps of the unbatched form (each view its own "
                         "graph-replayed plan, run one after another) for comparison (0: skip)")
    ap.add_argument("--batched-workload", default="batched_16views_1m",
                    help="the many-view leg reported beside the headline line: a workload of "
                         "several uneven views rendered as one batch ('none' to skip)")
    ap.add_argument("--batched-tile", default=BATCHED_TUNED["tile"],
                    help="tile of the many-view leg (its autotuned choice by default)")
    ap.add_argument("--batched-schedule", type=int, default=BATCHED_TUNED["schedule"])
    ap.add_argument("--batched-batch", type=int, default=BATCHED_TUNED["batch"])
    ap.add_argument("--batched-wave", type=int, default=BATCHED_TUNED["wave_w"])
    ap.add_argument("--batched-lane-masks", type=int, default=BATCHED_TUNED["lane_masks"])
    return ap.parse_args()


def depth_ablation(params, views, settings, reps: int, dev):
    """Forward kernels in both depth modes (HIP events around the library's
    launches) and the difference of the expected-depth maps over pixels with
    alpha > 0.5."""
    import dataclasses

    import torch

    from paper_2406_01467_amd import _lib
    from paper_2406_01467_amd.raster import Rasterizer
    res = {}
    depth = {}
    for name, mode in (("affine", _lib.RADE_DEPTH_AFFINE), ("exact", _lib.RADE_DEPTH_EXACT)):
        st = dataclasses.replace(settings, depth_mode=mode)
        rast = Rasterizer(views, st, dev)
        with torch.no_grad():
            maps = rast.forward(*params)
            torch.cuda.synchronize()
            ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(reps)] for k in ("project", "render_fwd")}
            kid = {"project": _lib.RADE_KERNEL_PROJECT, "render_fwd": _lib.RADE_KERNEL_RENDER_FWD}
            for lst in ev.values():
                for a, b in lst:
                    a.record()
                    b.record()
            torch.cuda.synchronize()
            for i in range(reps):
                for k in ev:
                    _lib.rade_set_kernel_events(kid[k], *ev[k][i])
                maps = rast.forward(*params)
            torch.cuda.synchronize()
            for k in ev:
                _lib.rade_set_kernel_events(kid[k], None, None)
        res[name] = {k: float(np.mean([a.elapsed_time(b) for a, b in ev[k]])) for k in ev}
        depth[name] = (maps.depth, maps.alpha)
    P = sum(v.width * v.height for v in views)
    da, alpha = depth["affine"]
    de, _ = depth["exact"]
    cov = torch.cat([alpha[o: o + v.width * v.height] > 0.5 for o, v in
                     zip(np.cumsum([0] + [v.width * v.height for v in views[:-1]]), views)])
    ea = torch.cat([da[2 * o: 2 * o + v.width * v.height] for o, v in
                    zip(np.cumsum([0] + [v.width * v.height for v in views[:-1]]), views)])
    ee = torch.cat([de[2 * o: 2 * o + v.width * v.height] for o, v in
                    zip(np.cumsum([0] + [v.width * v.height for v in views[:-1]]), views)])
    rel = ((ee - ea).abs() / ea.abs().clamp_min(1e-12))[cov]
    res["covered_pixels"] = int(cov.sum().item())
    res["expected_depth_rel_diff_mean"] = float(rel.mean().item()) if rel.numel() else None
    res["expected_depth_rel_diff_p99"] = (float(torch.quantile(rel.float(), 0.99).item())
                                          if rel.numel() else None)
    res["pixels"] = P
    return res


def mesh_extraction(scene, views, settings, grid: int, dev, reps: int = 3):
    """TSDF fusion of the views' median depth into a grid^3 box over the
    scene (2-98 percentile of the means) and Marching Cubes of its zero
    level, timed; HBM rates against the algorithmic bytes."""
    import torch

    from paper_2406_01467_amd.mesh import marching_cubes
    from paper_2406_01467_amd.raster import Rasterizer
    from paper_2406_01467_amd.tsdf import tsdf_fuse
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    rast = Rasterizer(views, settings, dev)
    with torch.no_grad():
        maps = rast.forward(t(scene.means), t(scene.scales), t(scene.quats),
                            t(scene.opacities), t(scene.sh.reshape(scene.n, -1)))
    lo = np.percentile(scene.means, 2, axis=0)
    hi = np.percentile(scene.means, 98, axis=0)
    voxel = float((hi - lo).max() / grid)
    dims = tuple(min(grid, int(np.ceil(e / voxel)) + 1) for e in (hi - lo))
    origin = lo.astype(np.float64)
    trunc = 4 * voxel
    nvox = int(np.prod(dims))
    tsdf, weight = tsdf_fuse(rast, maps.depth, origin, voxel, dims, trunc)
    verts, tris = marching_cubes(tsdf, weight, origin, voxel)  # sizes the outputs
    cap = (verts.shape[0], tris.shape[0])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        tsdf, weight = tsdf_fuse(rast, maps.depth, origin, voxel, dims, trunc)
    e1.record()
    torch.cuda.synchronize()
    fuse_ms = e0.elapsed_time(e1) / reps
    tm = time.perf_counter()
    for _ in range(reps):
        verts, tris = marching_cubes(tsdf, weight, origin, voxel, capacity=cap)
    torch.cuda.synchronize()
    mc_ms = 1e3 * (time.perf_counter() - tm) / reps
    P = rast.total_pixels
    fuse_bytes = 8 * nvox + 4 * P  # grid written once, median depth read once
    mc_bytes = 8 * nvox + 12 * verts.shape[0] + 12 * tris.shape[0]
    return {"grid": list(dims), "voxels": nvox, "views": len(views), "voxel": voxel,
            "seen_fraction": float((weight > 0).float().mean().item()),
            "tsdf_fuse_ms": fuse_ms,
            "tsdf_fuse_hbm": {"bound": "hbm", "algorithmic_bytes": fuse_bytes,
                              "achieved_GBs": fuse_bytes / (fuse_ms * 1e-3) / 1e9,
                              "peak_GBs": PEAK_HBM_GBS,
                              "frac": fuse_bytes / (fuse_ms * 1e-3) / 1e9 / PEAK_HBM_GBS},
            "marching_cubes_ms": mc_ms, "vertices": int(verts.shape[0]),
            "triangles": int(tris.shape[0]),
            "marching_cubes_hbm": {"bound": "hbm", "algorithmic_bytes": mc_bytes,
                                   "achieved_GBs": mc_bytes / (mc_ms * 1e-3) / 1e9,
                                   "peak_GBs": PEAK_HBM_GBS,
                                   "frac": mc_bytes / (mc_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                   "note": "wall time including the count read-back"}}


def cpu_baseline(scene, views, settings, npix: int, seed: int = 0):
    """FP64 oracle fwd+bwd on a bounded random pixel sample of view 0."""
    import oracle
    st = oracle.settings(sh_degree=settings.sh_degree, dilation=settings.dilation,
                         near=settings.near_plane, alpha_min=settings.alpha_min,
                         alpha_max=settings.alpha_max, t_min=settings.t_min,
                         power_cut=settings.power_cut, fov_clamp=settings.fov_clamp,
                         degenerate=settings.degenerate, bg=settings.bg)
    oracle.build()
    v = views[0]
    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(v.pixels, npix, replace=False)).astype(np.int64)
    t0 = time.perf_counter()
    rec, rect, flags = oracle.project(st, [v], scene)
    out = oracle.render(st, v, rec[0], flags[0], pix)
    t1 = time.perf_counter()
    g = rng.normal(size=(npix, 9))
    gP = oracle.render_bwd(st, v, rec[0], flags[0], g, pix)
    oracle.project_bwd(st, [v], scene, gP[None])
    t2 = time.perf_counter()
    blends = int(out["count"].sum())
    secs = t2 - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": blends / secs,
        "unit": "blends/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{npix} random pixels of view 0 of the same workload, fwd+bwd "
                   f"(projection of all {scene.n} Gaussians, brute-force blending over "
                   f"all of them per pixel, adjoint): {secs:.1f} s, fwd {t1 - t0:.1f} s"),
        "ms_per_view_extrapolated": 1e3 * secs * v.pixels / npix,
    }


def count_pass(views, settings, params, dev):
    """Blends, evaluations and pairs of one forward (deterministic for fixed
    inputs; counted with the default wave shape, which the blend count does
    not depend on)."""
    import torch

    from paper_2406_01467_amd.raster import Rasterizer
    with torch.no_grad():
        counter = Rasterizer(views, dataclasses.replace(settings, wave_w=0, batch=0, lane_masks=0),
                             dev)
        maps = counter.forward(*params, want_count=True, want_evals=True)
        torch.cuda.synchronize()
        blends = int(maps.count.sum().item())
        evals = int(maps.evals.to(torch.int64).sum().item())
        pairs = int(maps.state.n_pairs)
        del maps
    return blends, evals, pairs


def time_plan(plan, steps: int, warmup: int):
    """Replay a captured plan: wall ms per step and per-step HIP-event ms."""
    import torch
    plan.step()  # capture, replay, grow on overflow
    for _ in range(warmup):
        plan.replay()
    # per-step HIP events on the replay stream (recorded between replays, no
    # host synchronisation inside the timed window)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        plan.replay()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if plan.overflowed():
        raise RuntimeError("pair capacity overflow during the timed replays")
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return 1e3 * (t1 - t0) / steps, per


def kernel_times(plan, ksteps: int) -> dict:
    """Mean duration of each rasterizer kernel: HIP events the library
    records around each of its launches, on the stream it launches on, over
    steps enqueued eagerly."""
    import torch

    from paper_2406_01467_amd import _lib
    kinds = {"project": _lib.RADE_KERNEL_PROJECT, "render_fwd": _lib.RADE_KERNEL_RENDER_FWD,
             "render_bwd": _lib.RADE_KERNEL_RENDER_BWD,
             "project_bwd": _lib.RADE_KERNEL_PROJECT_BWD}
    events = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(ksteps)] for k in kinds}
    for lst in events.values():  # torch creates the HIP event on first record
        for a, b in lst:
            a.record()
            b.record()
    torch.cuda.synchronize()
    for i in range(ksteps):
        for k, kid in kinds.items():
            _lib.rade_set_kernel_events(kid, *events[k][i])
        plan.enqueue()
    torch.cuda.synchronize()
    for kid in kinds.values():
        _lib.rade_set_kernel_events(kid, None, None)
    return {k: float(np.mean([a.elapsed_time(b) for a, b in events[k]])) for k in kinds}


def unbatched_ms(views, settings, params, target, vcs, steps: int, recompute=False,
                 distortion=False, w_dist=0.0):
    """The same step unbatched: one graph-replayed plan per view, replayed
    one after another; ms for all views together."""
    import torch

    from paper_2406_01467_amd.batched import BatchedPlan
    from paper_2406_01467_amd.loss import make_grad_fn
    from paper_2406_01467_amd.raster import Rasterizer
    singles = []
    for vc, v in zip(vcs, views):
        r1 = Rasterizer([v], settings, params[0].device)
        tv = target[3 * vc.pix_offset: 3 * (vc.pix_offset + vc.width * vc.height)]
        p1 = BatchedPlan([v], settings, params, make_grad_fn(r1, tv, w_dist=w_dist),
                         recompute=recompute, distortion=distortion)
        p1.step()
        singles.append(p1)
    for p1 in singles:
        p1.replay()
    torch.cuda.synchronize()
    tu = time.perf_counter()
    for _ in range(steps):
        for p1 in singles:
            p1.replay()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - tu) / steps
    if any(p1.overflowed() for p1 in singles):
        raise RuntimeError("pair capacity overflow in the unbatched plans")
    del singles
    return ms


def rooflines(kernel_ms: dict, blends: int, n: int, views: int, pairs: int, pixels: int,
              sh_degree: int, ms_step: float, workload: str, settings,
              distortion: bool = False) -> tuple:
    """(roofline object of the dominant render kernel, whole-step HBM
    roofline) from the algorithmic flop and byte counts above."""
    dom = max(("render_fwd", "render_bwd"), key=lambda k: kernel_ms[k])
    dur = kernel_ms[dom] * 1e-3
    achieved = blends * FLOPS_PER_BLEND[dom] / dur / 1e12
    kb = kernel_bytes(dom, n, views, pairs, pixels)
    meas = measured(dom, workload, settings, distortion)
    roof = {"bound": "alu", "kernel": dom, "achieved": achieved,
            "peak": PEAK_FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_NONPACKED_TFLOPS,
            "peak_packed_fp32": PEAK_FP32_TFLOPS,
            "frac_of_packed_peak": achieved / PEAK_FP32_TFLOPS,
            "traffic": None if meas is None else meas["fetch_bytes"] + meas["write_bytes"],
            "valu_issue": None if meas is None else meas["valu_issue"],
            "hbm": {"algorithmic_bytes": kb, "achieved_GBs": kb / dur / 1e9,
                    "peak_GBs": PEAK_HBM_GBS, "frac": kb / dur / 1e9 / PEAK_HBM_GBS}}
    sb = step_bytes(n, views, pairs, pixels, sh_degree)
    whole = {"algorithmic_bytes": sb, "floor_ms": sb / (PEAK_HBM_GBS * 1e9) * 1e3,
             "achieved_GBs": sb / (ms_step * 1e-3) / 1e9,
             "frac": sb / (PEAK_HBM_GBS * 1e9) / (ms_step * 1e-3)}
    return roof, whole


def batched_leg(args, params, scene_n: int, sh_degree: int, dev) -> dict:
    """The many-view workload as one batch (one launch per kernel over all
    views, graph-replayed) against the same views unbatched."""
    import torch

    import synth
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan
    from paper_2406_01467_amd.loss import make_grad_fn
    from paper_2406_01467_amd.raster import Rasterizer
    scene, views = synth.make_workload(args.batched_workload)
    if scene.n != scene_n:
        raise RuntimeError("the many-view leg renders the headline workload's scene")
    tw, th = (int(x) for x in args.batched_tile.split("x"))
    st = Settings(tile_w=tw, tile_h=th, sh_degree=sh_degree, schedule=args.batched_schedule,
                  batch=args.batched_batch, wave_w=args.batched_wave,
                  lane_masks=args.batched_lane_masks)
    V = len(views)
    target = torch.from_numpy(synth.random_targets(views, seed=7)["color"]).to(dev)
    rast = Rasterizer(views, st, dev)
    blends, evals, pairs = count_pass(views, st, params, dev)
    plan = BatchedPlan(views, st, params, make_grad_fn(rast, target))
    ms, per = time_plan(plan, args.steps, args.warmup)
    kms = kernel_times(plan, max(3, min(args.steps, 5)))
    del plan
    ub = None
    if args.unbatched_steps > 0:
        ub = unbatched_ms(views, st, params, target, rast.views_c, args.unbatched_steps)
    roof, whole = rooflines(kms, blends, scene.n, V, pairs, rast.total_pixels, sh_degree, ms,
                            args.batched_workload, st)
    return {"workload": args.batched_workload, "views": V,
            "sizes": [[v.width, v.height] for v in views], "pixels": rast.total_pixels,
            "tile": args.batched_tile, "schedule": st.schedule,
            "batch": st.batch or tw * th, "wave": f"{st.wave_w or 8}x{64 // (st.wave_w or 8)}",
            "lane_masks": st.lane_masks,
            "mode": "all views in one launch per kernel, whole fwd+bwd step replayed as one "
                    "HIP graph",
            "ms_per_step": ms, "ms_per_view": ms / V,
            "step_ms_percentiles": {"p10": float(np.percentile(per, 10)),
                                    "p50": float(np.percentile(per, 50)),
                                    "p90": float(np.percentile(per, 90))},
            "ms_per_view_unbatched": None if ub is None else ub / V,
            "unbatched_mode": "one graph-replayed plan per view, replayed one after another",
            "blends_per_s": blends / (ms * 1e-3), "blends_per_view": blends / V,
            "pairs_per_view": pairs / V, "evals_per_blend": evals / max(1, blends),
            "kernel_ms": kms, "roofline": roof, "hbm_roofline_whole_step": whole}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan, autotune
    from paper_2406_01467_amd.loss import W_DIST, make_grad_fn, torch_loss
    from paper_2406_01467_amd.raster import Rasterizer, render

    dev = torch.device("cuda:0")
    scene, views = synth.make_workload(args.workload)
    tw, th = (16, 16) if args.tile == "auto" else (int(x) for x in args.tile.split("x"))
    settings = Settings(tile_w=tw, tile_h=th, sh_degree=scene.sh_degree, schedule=args.schedule,
                        lane_masks=args.lane_masks)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    params = [t(scene.means), t(scene.scales), t(scene.quats), t(scene.opacities),
              t(scene.sh.reshape(scene.n, -1))]
    target = torch.from_numpy(synth.random_targets(views, seed=7)["color"]).to(dev)
    V = len(views)

    w_dist = W_DIST if args.distortion else 0.0
    timings = {}
    if args.tile == "auto":
        probe = Rasterizer(views, settings, dev)
        settings, timings = autotune(views, params, settings,
                                     make_grad_fn(probe, target, w_dist=w_dist),
                                     distortion=args.distortion)
    rast = Rasterizer(views, settings, dev)
    blends, evals, pairs = count_pass(views, settings, params, dev)

    grad_fn = make_grad_fn(rast, target, w_dist=w_dist)
    torch.cuda.synchronize()
    mem_base = torch.cuda.memory_allocated()
    plan = BatchedPlan(views, settings, params, grad_fn, recompute=args.recompute,
                       distortion=args.distortion)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()  # the construction's sizing pass left out
    ms_step, per_step = time_plan(plan, args.steps, args.warmup)
    kernel_ms = kernel_times(plan, max(3, min(args.steps, 10)))
    loss_val = [float(x) for x in grad_fn.loss.cpu()]
    # device memory the plan (its buffers and workspaces) holds at the peak of
    # its steps
    peak_mem = int(torch.cuda.max_memory_allocated() - mem_base)
    del plan

    # several views: the same step unbatched for comparison with the batch
    ub_ms = None
    if V > 1 and args.unbatched_steps > 0:
        ub_ms = unbatched_ms(views, settings, params, target, rast.views_c,
                             args.unbatched_steps, args.recompute, args.distortion, w_dist)

    # the eager autograd path (user-facing API, torch loss) for comparison
    eager_ms = None
    if args.eager_steps > 0:
        leaves = [p.detach().clone().requires_grad_(True) for p in params]

        def eager_step():
            for p in leaves:
                p.grad = None
            outs = render(rast, *leaves, recompute=args.recompute, distortion=args.distortion)
            torch_loss(*outs[:4], target, rast.views_c,
                       distortion=outs[4] if args.distortion else None,
                       w_dist=w_dist).backward()

        for _ in range(2):
            eager_step()
        torch.cuda.synchronize()
        te = time.perf_counter()
        for _ in range(args.eager_steps):
            eager_step()
        torch.cuda.synchronize()
        eager_ms = 1e3 * (time.perf_counter() - te) / args.eager_steps
        del leaves

    value = blends / (ms_step * 1e-3)
    roof, whole = rooflines(kernel_ms, blends, scene.n, V, pairs, rast.total_pixels,
                            scene.sh_degree, ms_step, args.workload, settings, args.distortion)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "blends/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_view": ms_step / V,
        "step_ms_percentiles": {"p10": float(np.percentile(per_step, 10)),
                                "p50": float(np.percentile(per_step, 50)),
                                "p90": float(np.percentile(per_step, 90))},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "gaussians": scene.n, "views": V,
                   "pixels": rast.total_pixels, "sh_degree": scene.sh_degree,
                   "tile": f"{settings.tile_w}x{settings.tile_h}",
                   "wave": f"{settings.wave_w or 8}x{64 // (settings.wave_w or 8)}",
                   "batch": settings.batch or settings.tile_w * settings.tile_h,
                   "lane_masks": settings.lane_masks,
                   "schedule": settings.schedule,
                   "loss": "L1 colour + 5 x normal consistency (Eq. 24, median depth)" +
                           (" + 100 x depth distortion (Eq. 23)" if args.distortion else ""),
                   "mode": "whole fwd+bwd step replayed as one HIP graph",
                   "recompute_splats": bool(args.recompute)},
        "roofline": roof,
        "blends_per_view": blends / V,
        "pairs_per_view": pairs / V,
        "evals_per_blend": evals / max(1, blends),
        "kernel_ms": kernel_ms,
        "ms_per_view_eager_autograd": None if eager_ms is None else eager_ms / V,
        "ms_per_view_unbatched": None if ub_ms is None else ub_ms / V,
        "hbm_roofline_whole_step": whole,
        "loss": loss_val,
    }
    if peak_mem is not None:
        line["peak_memory_bytes"] = peak_mem
    if timings:
        line["autotune_ms"] = timings
    if args.batched_workload != "none" and V == 1:
        line["batched"] = batched_leg(args, params, scene.n, scene.sh_degree, dev)
    if args.depth_ablation > 0:
        line["depth_ablation"] = depth_ablation(params, views, settings, args.depth_ablation, dev)
    if args.mesh_grid > 0:
        line["mesh_extraction"] = mesh_extraction(scene, views, settings, args.mesh_grid, dev)
    if args.cpu_pixels > 0:
        line["cpu_baseline"] = cpu_baseline(scene, views, settings, args.cpu_pixels)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
