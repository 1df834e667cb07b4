#!/usr/bin/env python3
"""Benchmark of the RaDe-GS rasterizer hot path on one MI355X.

One step = one forward + backward pass of the whole path (projection with SH,
binning + depth/tile sort, tile rasterizer forward, the loss, rasterizer
backward, projection backward) over one view of the 1,000,000-Gaussian,
1600x1064 scene (64 anisotropic clusters at distance 2..20, SH degree 3), with
the loss L1(colour, target) + 5 * mean(alpha - N . n~) over interior pixels,
n~ the camera-facing normal of the back-projected median-depth map (not
detached).  Inputs are seeded synthetic and resident in HBM before timing.

Prints one JSON line: metric / value (splat-pixel blends per second) /
ms_per_step (fwd+bwd milliseconds per view), the roofline of the dominant
kernel from HIP events recorded around its launches inside the timed region,
and the FP64 CPU oracle timed on a bounded pixel sample.
"""
from __future__ import annotations

import argparse
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
W_NORMAL = 5.0                # normal-consistency weight (Sec. 4.1)

# Algorithmic FP32 operations per blended (pixel, splat) pair, counted from
# the method's arithmetic (FMA = 2): forward = offset (2), quadratic form (8),
# exp (1), alpha (1), 1-alpha and T (2), weight (1), colour (6), depth plane
# (4) and its blend (2), normal (6), alpha sum (1) = 34; backward = the same
# alpha (14), T recovery (2), weight (1), depth plane (4), upstream dot
# product (17), d alpha (4), running sum (2), depth grad (3), d power (2),
# centre grads (8), conic grads (7), opacity (1), colour (3), depth/plane (3),
# normal (3) = 74.
FLOPS_PER_BLEND_FWD = 34
FLOPS_PER_BLEND_BWD = 74
# Algorithmic HBM bytes (minimum traffic), per Gaussian, pair and pixel:
# params read 236 B (SH degree 3) twice (fwd, bwd), splat write 80 + read 80,
# tile count 4+4, splat-gradient record write+read 128, parameter grads 236;
# per pair: emit 8, sort 2 passes x 16, ranges 4, gather fwd 84, gather bwd 84;
# per pixel: maps + state 52 B written, read 52 + upstream grads 36.
BYTES_PER_GAUSSIAN = 236 * 2 + 80 * 2 + 8 + 128 + 236
BYTES_PER_PAIR = 8 + 32 + 4 + 84 + 84
BYTES_PER_PIXEL = 52 + 52 + 36


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="plain_1600x1064_1m")
    ap.add_argument("--tile", default="16x16", help="WxH, or 'auto' (batched mode)")
    ap.add_argument("--batched", action="store_true",
                    help="graph-replayed batched path over all views of the workload")
    ap.add_argument("--cpu-pixels", type=int, default=4096,
                    help="pixels of the oracle's CPU-baseline sample (0: skip)")
    ap.add_argument("--recompute", action="store_true",
                    help="keep no splats for the backward pass")
    return ap.parse_args()


def loss_fn(color, depth, normal, alpha, target, views_c):
    import torch
    import torch.nn.functional as F
    total = color.new_zeros(())
    for vc in views_c:
        H, W, o = vc.height, vc.width, vc.pix_offset
        P = H * W
        C = color[3 * o: 3 * o + 3 * P].view(3, H, W)
        D = depth[2 * o: 2 * o + 2 * P].view(2, H, W)[1]
        Nm = normal[3 * o: 3 * o + 3 * P].view(3, H, W)
        A = alpha[o: o + P].view(H, W)
        T = target[3 * o: 3 * o + 3 * P].view(3, H, W)
        l_c = (C - T).abs().mean()
        u = (torch.arange(W, device=C.device, dtype=C.dtype) + 0.5 - vc.cx) / vc.fx
        v = (torch.arange(H, device=C.device, dtype=C.dtype) + 0.5 - vc.cy) / vc.fy
        X = torch.stack([D * u[None, :], D * v[:, None], D], 0)
        du = X[:, 1:-1, 2:] - X[:, 1:-1, :-2]
        dv = X[:, 2:, 1:-1] - X[:, :-2, 1:-1]
        n = F.normalize(torch.cross(du, dv, dim=0), dim=0)
        facing = torch.where((n * X[:, 1:-1, 1:-1]).sum(0) > 0, -1.0, 1.0)
        n = n * facing
        l_n = (A[1:-1, 1:-1] - (Nm[:, 1:-1, 1:-1] * n).sum(0)).mean()
        total = total + l_c + W_NORMAL * l_n
    return total


def make_grad_fn(target, views_c):
    """Upstream gradients of the benchmark loss with respect to the maps,
    using only elementwise torch ops (safe inside a HIP graph: no reductions,
    no host synchronisation).  Per view: L1 colour mean + W_NORMAL x mean over
    interior pixels of (alpha - N . n~), n~ from the median depth."""
    import torch

    weights = []
    for vc in views_c:
        H, W = vc.height, vc.width
        weights.append((1.0 / (3 * H * W), W_NORMAL / ((H - 2) * (W - 2))))

    def grad_fn(maps):
        color, depth = maps["color"], maps["depth"]
        normal, alpha = maps["normal"], maps["alpha"]
        dC = torch.zeros_like(color)
        dD = torch.zeros_like(depth)
        dN = torch.zeros_like(normal)
        dA = torch.zeros_like(alpha)
        for vc, (wc, wn) in zip(views_c, weights):
            H, W, o = vc.height, vc.width, vc.pix_offset
            P = H * W
            C = color[3 * o: 3 * o + 3 * P]
            T = target[3 * o: 3 * o + 3 * P]
            dC[3 * o: 3 * o + 3 * P] = torch.sign(C - T) * wc
            with torch.enable_grad():
                D = depth[2 * o + P: 2 * o + 2 * P].view(H, W).detach().requires_grad_(True)
                Nm = normal[3 * o: 3 * o + 3 * P].view(3, H, W)[:, 1:-1, 1:-1]
                u = (torch.arange(W, device=D.device, dtype=D.dtype) + 0.5 - vc.cx) / vc.fx
                v = (torch.arange(H, device=D.device, dtype=D.dtype) + 0.5 - vc.cy) / vc.fy
                X = torch.stack([D * u[None, :], D * v[:, None], D], 0)
                du = X[:, 1:-1, 2:] - X[:, 1:-1, :-2]
                dv = X[:, 2:, 1:-1] - X[:, :-2, 1:-1]
                cx = du[1] * dv[2] - du[2] * dv[1]
                cy = du[2] * dv[0] - du[0] * dv[2]
                cz = du[0] * dv[1] - du[1] * dv[0]
                inv = torch.rsqrt(cx * cx + cy * cy + cz * cz + 1e-24)
                Xc = X[:, 1:-1, 1:-1]
                facing = torch.where(cx * Xc[0] + cy * Xc[1] + cz * Xc[2] > 0, -1.0, 1.0)
                s = facing * inv
                ndot = (Nm[0] * cx + Nm[1] * cy + Nm[2] * cz) * s
                (gD,) = torch.autograd.grad(ndot, D, grad_outputs=torch.full_like(ndot, -wn))
            dD[2 * o + P: 2 * o + 2 * P] = gD.reshape(-1)
            dN[3 * o: 3 * o + 3 * P].view(3, H, W)[:, 1:-1, 1:-1] = (
                -wn * s * torch.stack([cx, cy, cz], 0)).detach()
            dA[o: o + P].view(H, W)[1:-1, 1:-1] = wn
        return dC, dD, dN, dA

    return grad_fn


def run_batched(args, scene, views, settings, params, tgt, dev):
    """Graph-replayed batched fwd+bwd (autotuned) vs the plain per-view path."""
    import torch
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan, autotune
    from paper_2406_01467_amd.raster import Rasterizer, render

    probe = Rasterizer(views, settings, dev)
    grad_fn = make_grad_fn(tgt, probe.views_c)
    raw = [p.detach() for p in params]
    if args.tile == "auto":
        best, timings = autotune(views, raw, settings, grad_fn, reps=3)
    else:
        best, timings = settings, {}
    plan = BatchedPlan(views, best, raw, grad_fn)
    plan.step()
    with torch.no_grad():
        rast = Rasterizer(views, best, dev)
        maps = rast.forward(*raw, want_count=True)
        torch.cuda.synchronize()
        blends = int(maps.count.sum().item())
        pairs = int(maps.state.n_pairs)
        del maps, rast
    for _ in range(args.warmup):
        plan.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert not plan.overflowed()
    ms_step = 1e3 * (t1 - t0) / args.steps
    # the unbatched plain form: one eager call sequence per view
    plain = [Rasterizer([v], Settings(**{**settings.__dict__, "schedule": 0}), dev) for v in views]
    gfns = [make_grad_fn(tgt[3 * vc.pix_offset: 3 * vc.pix_offset + 3 * vc.width * vc.height],
                         [r.views_c[0]]) for r, vc in zip(plain, probe.views_c)]

    def plain_step():
        for r, gf in zip(plain, gfns):
            m = r.forward(*raw)
            mp = dict(color=m.color, depth=m.depth, normal=m.normal, alpha=m.alpha)
            r.backward(m.state, *raw, *gf(mp))

    for _ in range(max(1, args.warmup // 2)):
        plain_step()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(max(2, args.steps // 4)):
        plain_step()
    torch.cuda.synchronize()
    ms_plain = 1e3 * (time.perf_counter() - t2) / max(2, args.steps // 4)
    return best, timings, ms_step, ms_plain, blends, pairs


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
    gP = gP[None]
    oracle.project_bwd(st, [v], scene, gP)
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
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_2406_01467_amd import Settings, _lib
    from paper_2406_01467_amd.raster import Rasterizer, render

    dev = torch.device("cuda:0")
    tw, th = (16, 16) if args.tile == "auto" else (int(x) for x in args.tile.split("x"))
    scene, views = synth.make_workload(args.workload)
    settings = Settings(tile_w=tw, tile_h=th, sh_degree=scene.sh_degree)
    rast = Rasterizer(views, settings, dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    params = [t(scene.means), t(scene.scales), t(scene.quats), t(scene.opacities),
              t(scene.sh.reshape(scene.n, -1))]
    for p in params:
        p.requires_grad_(True)
    tgt = torch.from_numpy(synth.random_targets(views, seed=7)["color"]).to(dev)

    if args.batched:
        best, timings, ms_step, ms_plain, blends, pairs = run_batched(
            args, scene, views, settings, params, tgt, dev)
        V = len(views)
        line = {
            "metric": METRIC, "value": blends / (ms_step * 1e-3), "unit": "blends/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_step / V, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": args.workload, "gaussians": scene.n, "views": V,
                       "pixels": sum(v.pixels for v in views), "sh_degree": scene.sh_degree,
                       "tile": f"{best.tile_w}x{best.tile_h}", "schedule": best.schedule,
                       "mode": "batched, one launch per kernel, HIP graph replay"},
            "ms_per_view_unbatched_plain": ms_plain / V,
            "speedup_vs_plain": ms_plain / ms_step,
            "autotune_ms": timings, "blends_per_step": blends, "pairs_per_step": pairs,
        }
        print(json.dumps(line), flush=True)
        return

    # blends per step (deterministic for fixed inputs) and pair count
    with torch.no_grad():
        maps = rast.forward(*[p.detach() for p in params], want_count=True)
        torch.cuda.synchronize()
        blends = int(maps.count.sum().item())
        pairs = int(maps.state.n_pairs)
        del maps

    def step():
        for p in params:
            p.grad = None
        color, depth, normal, alpha = render(rast, *params, recompute=args.recompute)
        loss = loss_fn(color, depth, normal, alpha, tgt, rast.views_c)
        loss.backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    kinds = {"render_fwd": _lib.RADE_KERNEL_RENDER_FWD, "render_bwd": _lib.RADE_KERNEL_RENDER_BWD,
             "project": _lib.RADE_KERNEL_PROJECT, "project_bwd": _lib.RADE_KERNEL_PROJECT_BWD}
    events = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)] for k in kinds}
    for pairs_k in events.values():  # torch creates the HIP event on first record
        for a, b in pairs_k:
            a.record()
            b.record()
    # bracket: device idle, then time exactly K steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        for k, kid in kinds.items():
            _lib.rade_set_kernel_events(kid, *events[k][i])
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for kid in kinds.values():
        _lib.rade_set_kernel_events(kid, None, None)
    kernel_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in events[k]])) for k in kinds}

    ms_step = 1e3 * (t1 - t0) / args.steps
    V = len(views)
    ms_view = ms_step / V
    value = blends / (ms_step * 1e-3)
    dom = max(("render_fwd", "render_bwd"), key=lambda k: kernel_ms[k])
    flops = blends * (FLOPS_PER_BLEND_BWD if dom == "render_bwd" else FLOPS_PER_BLEND_FWD)
    achieved = flops / (kernel_ms[dom] * 1e-3) / 1e12
    alg_bytes = (BYTES_PER_GAUSSIAN * scene.n * V + BYTES_PER_PAIR * pairs +
                 BYTES_PER_PIXEL * rast.total_pixels)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "blends/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_view,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "gaussians": scene.n, "views": V,
                   "width": views[0].width, "height": views[0].height,
                   "sh_degree": scene.sh_degree, "tile": args.tile,
                   "loss": "L1 colour + 5 x normal consistency (median depth)",
                   "recompute_splats": bool(args.recompute)},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None},
        "blends_per_view": blends / V,
        "pairs_per_view": pairs / V,
        "kernel_ms": kernel_ms,
        "hbm_roofline_whole_step": {"algorithmic_bytes": alg_bytes,
                                    "floor_ms": alg_bytes / (PEAK_HBM_GBS * 1e9) * 1e3,
                                    "frac": alg_bytes / (PEAK_HBM_GBS * 1e9) / (ms_step * 1e-3)},
    }
    if args.cpu_pixels > 0:
        line["cpu_baseline"] = cpu_baseline(scene, views, settings, args.cpu_pixels)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
