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
fwd+bwd milliseconds per step (all views), ms_per_view = the same per view; roofline of the dominant kernel (HIP events
recorded by the library around its launches); the eager autograd path
(torch.autograd.Function + torch loss) for comparison; the FP64 CPU oracle
timed on a bounded pixel sample.
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
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak (packed)
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
# Algorithmic HBM bytes (minimum traffic), per Gaussian and view, per pair
# and per pixel: params read 236 B (SH degree 3) in the forward and again in
# the backward, splat write 80 + read 80, tile count 4+4, splat-gradient
# record write+read 128, parameter gradients 236; per pair: emit 8, two sort
# passes x 16, ranges 4, gather fwd 84, gather bwd 84; per pixel: maps and
# state written 52, read back 52, upstream gradients 36.
BYTES_PER_GAUSSIAN = 236 * 2 + 80 * 2 + 8 + 128 + 236
BYTES_PER_PAIR = 8 + 32 + 4 + 84 + 84
BYTES_PER_PIXEL = 52 + 52 + 36

# HBM traffic of one launch of the dominant kernel, from two rocprofv3 --pmc
# runs of paper_2406_01467_amd/profile_step.py (FETCH_SIZE, then WRITE_SIZE,
# KiB per dispatch), each scaled by what the counter reads for a copy kernel
# of known size (FETCH_SIZE reads half of the bytes a plain copy moves,
# WRITE_SIZE all of them).  Valid only for the kernel sources it was measured
# on (SHA-1 of render.hip + common.hpp) and for the 1600x1064 / 1M workload
# in the launch configuration it was measured in (tile, schedule, wave shape,
# batch); reported as null otherwise.
MEASURED_TRAFFIC = {"kernel": "render_bwd", "workload": "plain_1600x1064_1m", "tile": "16x16",
                    "schedule": 1, "wave_w": 0, "batch": 0,
                    "sources_sha1": "b0a199b33eccdf631439c5b0de8c37afe06f6e31",
                    "fetch_bytes": 375196176, "write_bytes": 154785088,
                    "profile": "profiles/kernels_1600x1064_1m_pmc.md"}


def _render_sources_sha1() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in ("render.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2406_01467_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str, settings):
    t = MEASURED_TRAFFIC
    tile = f"{settings.tile_w}x{settings.tile_h}"
    if (t is None or t["kernel"] != kernel or t["workload"] != workload or t["tile"] != tile
            or t["schedule"] != settings.schedule or t["wave_w"] != settings.wave_w
            or t["batch"] != settings.batch or t["sources_sha1"] != _render_sources_sha1()):
        return None
    return t["fetch_bytes"] + t["write_bytes"]


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_2406_01467_amd import Settings, _lib
    from paper_2406_01467_amd.batched import BatchedPlan, autotune
    from paper_2406_01467_amd.loss import W_DIST, make_grad_fn, torch_loss
    from paper_2406_01467_amd.raster import Rasterizer, render

    dev = torch.device("cuda:0")
    scene, views = synth.make_workload(args.workload)
    tw, th = (16, 16) if args.tile == "auto" else (int(x) for x in args.tile.split("x"))
    settings = Settings(tile_w=tw, tile_h=th, sh_degree=scene.sh_degree, schedule=args.schedule)
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

    # blends and pairs per step (deterministic for fixed inputs; the blend
    # count is compiled for the default wave shape, and does not depend on it)
    with torch.no_grad():
        counter = Rasterizer(views, dataclasses.replace(settings, wave_w=0, batch=0), dev)
        maps = counter.forward(*params, want_count=True)
        torch.cuda.synchronize()
        blends = int(maps.count.sum().item())
        pairs = int(maps.state.n_pairs)
        del maps

    grad_fn = make_grad_fn(rast, target, w_dist=w_dist)
    plan = BatchedPlan(views, settings, params, grad_fn, recompute=args.recompute,
                       distortion=args.distortion)
    plan.step()  # capture, replay, grow on overflow
    for _ in range(args.warmup):
        plan.replay()
    # per-step HIP events on the replay stream (recorded between replays, no
    # host synchronisation inside the timed window)
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ev[0].record()
    for i in range(args.steps):
        plan.replay()
        step_ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if plan.overflowed():
        raise RuntimeError("pair capacity overflow during the timed replays")
    ms_step = 1e3 * (t1 - t0) / args.steps
    per_step = np.array([step_ev[i].elapsed_time(step_ev[i + 1]) for i in range(args.steps)])

    # per-kernel durations: HIP events recorded by the library around each
    # launch, over the same steps enqueued eagerly on the same stream
    kinds = {"project": _lib.RADE_KERNEL_PROJECT, "render_fwd": _lib.RADE_KERNEL_RENDER_FWD,
             "render_bwd": _lib.RADE_KERNEL_RENDER_BWD,
             "project_bwd": _lib.RADE_KERNEL_PROJECT_BWD}
    ksteps = max(3, min(args.steps, 10))
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
    kernel_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in events[k]])) for k in kinds}

    # several views: the same step unbatched (one plan per view, replayed
    # one after another) for comparison with the one-launch-per-kernel batch
    unbatched_ms = None
    if V > 1 and args.unbatched_steps > 0:
        singles = []
        for vc, v in zip(rast.views_c, views):
            r1 = Rasterizer([v], settings, dev)
            tv = target[3 * vc.pix_offset: 3 * (vc.pix_offset + vc.width * vc.height)]
            p1 = BatchedPlan([v], settings, params, make_grad_fn(r1, tv, w_dist=w_dist),
                             recompute=args.recompute, distortion=args.distortion)
            p1.step()
            singles.append(p1)
        for p1 in singles:
            p1.replay()
        torch.cuda.synchronize()
        tu = time.perf_counter()
        for _ in range(args.unbatched_steps):
            for p1 in singles:
                p1.replay()
        torch.cuda.synchronize()
        unbatched_ms = 1e3 * (time.perf_counter() - tu) / args.unbatched_steps
        if any(p1.overflowed() for p1 in singles):
            raise RuntimeError("pair capacity overflow in the unbatched plans")
        del singles

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

    value = blends / (ms_step * 1e-3)
    dom = max(("render_fwd", "render_bwd"), key=lambda k: kernel_ms[k])
    achieved = blends * FLOPS_PER_BLEND[dom] / (kernel_ms[dom] * 1e-3) / 1e12
    alg_bytes = (BYTES_PER_GAUSSIAN * scene.n * V + BYTES_PER_PAIR * pairs +
                 BYTES_PER_PIXEL * rast.total_pixels)
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
                   "schedule": settings.schedule,
                   "loss": "L1 colour + 5 x normal consistency (Eq. 24, median depth)" +
                           (" + 100 x depth distortion (Eq. 23)" if args.distortion else ""),
                   "mode": "whole fwd+bwd step replayed as one HIP graph",
                   "recompute_splats": bool(args.recompute)},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(dom, args.workload, settings)},
        "blends_per_view": blends / V,
        "pairs_per_view": pairs / V,
        "kernel_ms": kernel_ms,
        "ms_per_view_eager_autograd": None if eager_ms is None else eager_ms / V,
        "ms_per_view_unbatched": None if unbatched_ms is None else unbatched_ms / V,
        "hbm_roofline_whole_step": {"algorithmic_bytes": alg_bytes,
                                    "floor_ms": alg_bytes / (PEAK_HBM_GBS * 1e9) * 1e3,
                                    "frac": alg_bytes / (PEAK_HBM_GBS * 1e9) / (ms_step * 1e-3)},
        "loss": [float(x) for x in grad_fn.loss.cpu()],
    }
    if timings:
        line["autotune_ms"] = timings
    if args.depth_ablation > 0:
        line["depth_ablation"] = depth_ablation(params, views, settings, args.depth_ablation, dev)
    if args.mesh_grid > 0:
        line["mesh_extraction"] = mesh_extraction(scene, views, settings, args.mesh_grid, dev)
    if args.cpu_pixels > 0:
        line["cpu_baseline"] = cpu_baseline(scene, views, settings, args.cpu_pixels)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
