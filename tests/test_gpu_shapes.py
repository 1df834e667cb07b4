"""Wave shapes (8x8, 16x4, 32x2 pixels per wavefront) and staging batches
(64..256 splats per round) of the render kernels: the maps are the same bits
whatever the shape (each pixel blends the same list in the same order), the
gradients equal up to the order of FP32 atomic additions, one tuned shape
matches the FP64 oracle, and the paths compiled for the default shape only
reject the others."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import compare_maps, device, grad_check, oracle_settings, say, to_dev

pytestmark = pytest.mark.gpu

KEYS = ("color", "depth", "normal", "alpha", "t_final", "last", "median")


def _settings(**kw):
    from paper_2406_01467_amd import Settings
    return Settings(**kw)


def _shapes(tw, th):
    """(wave width, staging batch, lane masks) of every shape the tile holds;
    lane masks on tiles of several 8x8 waves with one splat per thread."""
    out = []
    for ww in (8, 16, 32):
        if tw % ww or th % (64 // ww):
            continue
        for bt in (0, 64, 128, 256):
            out.append((ww, bt, 0))
    if tw * th > 64:
        out.append((8, 0, 1))
    return out


def _scene():
    scene = synth.make_scene_ball(6000, seed=101, centre=(0.0, 0.0, 3.0), radius=1.2,
                                  log_scale_mu=-3.2)
    return scene, [synth.identity_view(100, 70)]


@pytest.mark.parametrize("tile", [(16, 16), (32, 16), (16, 8), (8, 8), (16, 32)])
def test_maps_are_identical_across_shapes(tile):
    import torch
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene()
    params = to_dev(scene, dev)
    ref = None
    for ww, bt, lm in _shapes(*tile):
        rast = Rasterizer(views, _settings(sh_degree=3, tile_w=tile[0], tile_h=tile[1],
                                           wave_w=ww, batch=bt, lane_masks=lm), dev)
        maps = rast.forward(*params)
        torch.cuda.synchronize()
        got = {k: getattr(maps, k) if hasattr(maps, k) else getattr(maps.state, k) for k in KEYS}
        got = {k: v.cpu().numpy() for k, v in got.items()}
        if ref is None:
            ref = got
            continue
        for k in KEYS:
            assert np.array_equal(got[k].view(np.uint32), ref[k].view(np.uint32)), \
                (tile, ww, bt, lm, k)
    say(f"  tile {tile}: {len(_shapes(*tile))} shapes, identical maps")


def _grads(rast, maps, params, ups, dev):
    import torch
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    out = rast.backward(maps.state, *params, *(t(u) for u in ups))
    torch.cuda.synchronize()
    return [g.cpu().numpy().astype(np.float64) for g in out]


def test_gradients_agree_across_shapes():
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene()
    params = to_dev(scene, dev)
    rng = np.random.default_rng(102)
    P = views[0].pixels
    ups = [rng.normal(size=k * P).astype(np.float32) for k in (3, 2, 3, 1)]
    ref = None
    # 8x8 tiles and lane-mask shapes take the quadrant-group backward (one,
    # two or four 64-splat chunks per staging round)
    for tile in [(16, 16), (32, 16), (8, 8)]:
        for ww, bt, lm in _shapes(*tile):
            rast = Rasterizer(views, _settings(sh_degree=3, tile_w=tile[0], tile_h=tile[1],
                                               wave_w=ww, batch=bt, lane_masks=lm), dev)
            g = _grads(rast, rast.forward(*params), params, ups, dev)
            if ref is None:
                ref = g
                continue
            for a, b, name in zip(g, ref, ("means", "scales", "quats", "opacities", "sh")):
                rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
                # FP32 atomics add the per-wave partial sums in another grouping:
                # the bar of the recompute-vs-stored comparison
                assert rel <= 1e-5, (tile, ww, bt, lm, name, rel)


def test_backward_reads_the_forward_lane_masks():
    """Where the launch shape keeps lane masks, the forward stores them per
    (pair, 8x8 wave) and the backward reads them instead of recomputing: the
    gradients with and without that cache agree up to the order of the FP32
    atomic additions, and shapes without lane masks keep no cache."""
    import dataclasses
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene()
    params = to_dev(scene, dev)
    rng = np.random.default_rng(103)
    P = views[0].pixels
    ups = [rng.normal(size=k * P).astype(np.float32) for k in (3, 2, 3, 1)]
    cases = [((8, 8), 0, 0), ((8, 8), 256, 0), ((16, 16), 0, 1), ((32, 16), 0, 1),
             ((16, 8), 0, 1), ((16, 16), 0, 0)]
    for (tw, th), bt, lm in cases:
        rast = Rasterizer(views, _settings(sh_degree=3, tile_w=tw, tile_h=th, batch=bt,
                                           lane_masks=lm), dev)
        maps = rast.forward(*params)
        kept = maps.state.lane_masks
        waves = (tw // 8) * (th // 8) if (lm or (tw, th) == (8, 8)) else 0
        if waves == 0:
            assert kept is None, (tw, th, bt, lm)
            continue
        assert kept is not None and kept.numel() >= maps.state.n_pairs * waves
        # the cache holds masks of staged pairs: some pixels of each tile
        assert int((kept[: maps.state.n_pairs * waves] != 0).sum()) > 0
        g_cache = _grads(rast, maps, params, ups, dev)
        g_comp = _grads(rast, type("M", (), {"state": dataclasses.replace(maps.state,
                                                                          lane_masks=None)}),
                        params, ups, dev)
        for a, b, name in zip(g_cache, g_comp, ("means", "scales", "quats", "opacities", "sh")):
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            say(f"  {tw}x{th} batch {bt} lane masks {lm}: {name} cache vs computed {rel:.3g}")
            assert rel <= 1e-5, (tw, th, bt, lm, name, rel)


def test_tuned_shape_matches_the_oracle():
    import torch
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene = synth.make_scene_clusters(8000, seed=103, width=120, height=90, dist_range=(2, 6))
    views = [synth.identity_view(120, 90)] + synth.make_views_orbit(
        scene.means.mean(0), 5.0, 1, seed=104, sizes=[(77, 131)])
    s = _settings(sh_degree=3, tile_w=32, tile_h=16, wave_w=32, batch=64, bg=(0.25, 0.5, 1.0))
    rast = Rasterizer(views, s, dev)
    params = to_dev(scene, dev)
    maps = rast.forward(*params)
    torch.cuda.synchronize()
    _, _, _, outs = oracle.forward(oracle_settings(s), views, scene)
    nfrag = 0
    for vi in range(len(views)):
        g = {k: v.cpu().numpy() for k, v in maps.view_planes(rast, vi).items()}
        nfrag += compare_maps(g, outs[vi], check_int=False, label=f"32x2/64 view {vi}: ")
    assert nfrag <= max(2, 1e-2 * sum(v.pixels for v in views))
    rng = np.random.default_rng(105)
    P = rast.total_pixels
    ups = [rng.normal(size=k * P).astype(np.float32) for k in (3, 2, 3, 1)]
    got = _grads(rast, maps, params, ups, dev)
    gouts = []
    for vi, v in enumerate(views):
        o, Pv = rast.views_c[vi].pix_offset, v.pixels
        gg = np.zeros((Pv, 9))
        gg[:, 0:3] = ups[0][3 * o: 3 * o + 3 * Pv].reshape(3, Pv).T
        gg[:, 3:5] = ups[1][2 * o: 2 * o + 2 * Pv].reshape(2, Pv).T
        gg[:, 5:8] = ups[2][3 * o: 3 * o + 3 * Pv].reshape(3, Pv).T
        gg[:, 8] = ups[3][o: o + Pv]
        gouts.append(gg)
    st = oracle_settings(s)
    ref = oracle.backward(st, views, scene, gouts)
    scale = oracle.gradient_error_scale(st, views, scene, gouts)
    grad_check(dict(zip(("means", "scales", "quats", "opacities", "sh"), got)), ref, scale,
               "32x2 waves, batch 64")


def test_special_paths_need_the_default_shape():
    import torch
    from paper_2406_01467_amd import _lib
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene()
    params = to_dev(scene, dev)
    s = _settings(sh_degree=3, wave_w=16, batch=64)
    rast = Rasterizer(views, s, dev)
    for kw in (dict(want_count=True), dict(want_distortion=True)):
        with pytest.raises(_lib.RadeError) as ei:
            rast.forward(*params, **kw)
        assert ei.value.code == _lib.RADE_ERR_INVALID_ARG
    exact = Rasterizer(views, _settings(sh_degree=3, wave_w=16, batch=64, depth_mode=1), dev)
    with pytest.raises(_lib.RadeError):
        exact.forward(*params)
    maps = rast.forward(*params)
    P = rast.total_pixels
    z = lambda k: torch.zeros(k * P, device=dev)  # noqa: E731
    with pytest.raises(_lib.RadeError):
        rast.backward(maps.state, *params, z(3), z(2), z(3), z(1), d_distortion=z(1))
