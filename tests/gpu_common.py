"""Helpers of the GPU parity tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs, and compare."""
import os
import sys

import numpy as np
import pytest

import oracle


def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_01467_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        raise RuntimeError("librade.so missing: build before running GPU tests")
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_settings(s):
    return oracle.settings(sh_degree=s.sh_degree, dilation=s.dilation, near=s.near_plane,
                           alpha_min=s.alpha_min, alpha_max=s.alpha_max, t_min=s.t_min,
                           power_cut=s.power_cut, fov_clamp=s.fov_clamp,
                           degenerate=s.degenerate, bg=s.bg, tile=(s.tile_w, s.tile_h),
                           depth_exact=s.depth_mode == 1)


def to_dev(scene, dev):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    return (t(scene.means), t(scene.scales), t(scene.quats), t(scene.opacities),
            t(scene.sh.reshape(scene.n, scene.sh.shape[1] * 3)))


def gpu_forward(scene, views, settings, dev, keep=True):
    """Returns (rasterizer, maps, per-view numpy dicts)."""
    import torch
    from paper_2406_01467_amd.raster import Rasterizer
    rast = Rasterizer(views, settings, dev)
    params = to_dev(scene, dev)
    # the counting pass exists for the default wave shape and batch only
    count = settings.batch == 0 and settings.wave_w == 0 and settings.lane_masks == 0
    maps = rast.forward(*params, want_count=count, keep_splats=keep)
    torch.cuda.synchronize()
    per_view = []
    pair_ids = maps.state.pair_ids.cpu().numpy().astype(np.int64)
    ranges = maps.state.ranges.cpu().numpy().astype(np.int64).reshape(-1, 2)
    for vi, v in enumerate(views):
        d = {k: t.cpu().numpy() for k, t in maps.view_planes(rast, vi).items()}
        vc = rast.views_c[vi]
        H, W = v.height, v.width
        py, px = np.mgrid[0:H, 0:W]
        tile = vc.tile_offset + (py // settings.tile_h) * vc.tiles_x + px // settings.tile_w
        last = d["last"][0]
        lid = np.where(last >= 0, pair_ids[np.clip(ranges[tile, 0] + last, 0,
                                                    max(0, len(pair_ids) - 1))], -1)
        d["last_id"] = lid
        per_view.append(d)
    return rast, maps, per_view, params


def flat(a):
    return np.asarray(a).reshape(a.shape[0], -1) if a.ndim == 3 else a.reshape(-1)


def compare_maps(g, o, pixels=None, tol=1e-5, check_int=True, label=""):
    """g: GPU per-view dict (C,H,W); o: oracle dict for the pixel list (or all
    pixels).  Non-fragile pixels only.  Element-wise bound
    |x - x_ref| <= tol (|x_ref| + 1e-3 max|x_ref|), and for the normal
    components, whose terms cancel, tol (|x_ref| + 1e-3 max|x_ref| + alpha_ref).
    Integer maps exact.  Returns the number of fragile pixels."""
    frag = (o["fragile"] & 1) != 0
    keep = ~frag

    def gp(name, c=None):
        a = g[name]
        a = a.reshape(a.shape[0], -1)
        a = a if pixels is None else a[:, pixels]
        return a if c is None else a[c]

    alpha_ref = np.asarray(o["alpha"], np.float64)[keep]
    failures = []

    def check(got, ref, what, cancelling=False):
        got = np.asarray(got, np.float64)[keep]
        ref = np.asarray(ref, np.float64)[keep]
        if ref.size == 0:
            return
        floor = 1e-3 * np.abs(ref).max()
        if cancelling:
            # Sum of terms of both signs bounded by the blend weights: FP32
            # round-off scales with sum |w_i f_i| <= sum w_i = alpha.
            floor = floor + alpha_ref
        err = np.abs(got - ref)
        bound = tol * (np.abs(ref) + floor)
        bad = err > bound
        rel = err / (np.abs(ref) + floor + 1e-30)
        i = int(np.argmax(rel))
        if bad.any():
            failures.append(f"{label}{what}: {bad.sum()} of {bad.size} pixels beyond "
                            f"{tol}; worst rel {rel[i]:.3g} (ref {ref[i]:.6g} got {got[i]:.6g} "
                            f"alpha {alpha_ref[i]:.4g} err/alpha "
                            f"{err[i] / max(alpha_ref[i], 1e-30):.3g})")

    for c in range(3):
        check(gp("color", c), o["color"][:, c], f"color[{c}]")
        check(gp("normal", c), o["normal"][:, c], f"normal[{c}]", cancelling=True)
    check(gp("depth", 0), o["depth_exp"], "depth_exp")
    check(gp("depth", 1), o["depth_med"], "depth_med")
    check(gp("alpha", 0), o["alpha"], "alpha")
    check(gp("t_final", 0), o["t_final"], "t_final")
    if check_int:
        for name, ref in (("count", o["count"]), ("median", o["median_id"])):
            if name not in g:  # e.g. a batched plan renders no count map
                continue
            got = gp(name, 0)
            mism = (got != ref) & keep
            if mism.any():
                failures.append(f"{label}{name}: {mism.sum()} mismatching pixels")
        lid = g["last_id"].reshape(-1)
        lid = lid if pixels is None else lid[pixels]
        mism = (lid != o["last_id"]) & keep
        if mism.any():
            failures.append(f"{label}last_id: {mism.sum()} mismatching pixels")
    for f in failures:
        print(f, flush=True)
    assert not failures, failures
    return int(frag.sum())


def grad_check(got, ref, scale, label, tol=1e-4, normwise_tol=1e-5):
    """Per parameter group: norm-wise ||g - g_ref|| <= 1e-5 (||g_ref|| +
    0.1 ||S||), and element-wise |g - g_ref| <= 1e-4 (|g_ref| + 0.1 S), where
    S is the oracle's round-off scale of that element (sum over pixels of
    |term|, pushed through |d param / d splat quantity|).  A gradient element
    is a sum of per-pixel FP32 terms of both signs; its attainable accuracy
    is set by the size of the terms, not by their (possibly cancelling) sum:
    the element-wise bound allows 1e-5 S, about 170 units of FP32 round-off,
    and the norm-wise one the same floor over the group (on scenes of
    needle-like splats the scale gradients cancel to ~1/50 of S, and two
    orders of the FP32 atomic additions differ by 1e-5 of ||g_ref||)."""
    worst = {}
    for k in ref:
        r = np.asarray(ref[k], np.float64).reshape(ref[k].shape[0], -1)
        g = np.asarray(got[k], np.float64).reshape(r.shape)
        S = np.asarray(scale[k], np.float64).reshape(r.shape)
        if r.size == 0:
            continue
        aerr = np.abs(g - r)
        err = aerr / (np.abs(r) + 0.1 * S + 1e-30)
        nrm_plain = np.linalg.norm(g - r) / (np.linalg.norm(r) + 1e-30)
        nrm = np.linalg.norm(g - r) / (np.linalg.norm(r) + 0.1 * np.linalg.norm(S) + 1e-30)
        i = np.unravel_index(np.argmax(err), err.shape)
        worst[k] = (float(err.max()), float(nrm))
        # elements within the bar only thanks to the round-off floor: beyond
        # tol relative to |g_ref| but within tol (|g_ref| + 0.1 S)
        floor_only = (aerr > tol * np.abs(r)) & (aerr <= tol * (np.abs(r) + 0.1 * S))
        nz = int((r != 0).sum())
        rel_nz = aerr[r != 0] / np.abs(r[r != 0]) if nz else np.zeros(1)
        say(f"  grad {k}: normwise {nrm_plain:.3g} (with the 0.1 S floor {nrm:.3g}); worst elem {err[i]:.3g} (ref {r[i]:.4g} got "
            f"{g[i]:.4g}, scale {S[i]:.4g}); max |err|/S {np.max(aerr / (S + 1e-30)):.3g}; "
            f"{int(floor_only.sum())} of {r.size} elements pass only through the 0.1 S floor; "
            f"relative error of nonzero elements: median {np.median(rel_nz):.3g}, "
            f"99th pct {np.percentile(rel_nz, 99):.3g}")
    say(label, "gradient errors (element, normwise)", worst)
    for k, (w, n) in worst.items():
        assert w <= tol and n <= normwise_tol, (label, k, w, n)
