"""GPU parity of the HIP path (through the C ABI) with the FP64 oracle.

Maps: |x - x_ref| <= 1e-5 (|x_ref| + 1e-3 max|x_ref|) on every pixel that the
oracle does not flag as fragile (within FP32 reach of a discrete threshold),
integer maps (blend count, last and median Gaussian ids) exact there.
Normal components (terms of both signs) use alpha as an extra floor.
Projection fields 1e-5 relative; tile lists, keys and ranges bit-exact.
Gradients: norm-wise 1e-5 and element-wise 1e-4 with a floor, see gpu_common.grad_check."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import (compare_maps, device, gpu_forward, grad_check, oracle_settings, say,
                        to_dev)
from oracle_helpers import scene_from, view

pytestmark = pytest.mark.gpu


def _settings(**kw):
    from paper_2406_01467_amd import Settings
    return Settings(**kw)


def _workload(name, n=None, views=None):
    scene, vs = synth.make_workload(name, n=n)
    return scene, (views or vs)


# ---------------------------------------------------------------------------
# projection

def _gpu_splats(scene, views, s, dev):
    import torch
    from paper_2406_01467_amd.raster import Rasterizer
    from paper_2406_01467_amd import _lib
    rast = Rasterizer(views, s, dev)
    splats, tt, brec = rast.project(*to_dev(scene, dev))
    torch.cuda.synchronize()
    sp = splats.cpu().numpy().view(_lib.SPLAT_DTYPE).reshape(len(views), scene.n)
    br = brec.cpu().numpy().view(np.uint32).reshape(len(views), scene.n, 4)
    return sp, tt.cpu().numpy().reshape(len(views), scene.n), rast, br


@pytest.mark.parametrize("name,n", [("plain_64x64_1k", None), ("plain_800x800_200k", 20000),
                                    ("plain_1600x1064_1m", 30000)])
def test_project_parity(name, n):
    dev = device()
    scene, views = _workload(name, n)
    s = _settings(sh_degree=scene.sh_degree)
    say("project parity", name, scene.n)
    sp, tt, _, br = _gpu_splats(scene, views, s, dev)
    rec, rect, flags = oracle.project(oracle_settings(s), views, scene)
    R = oracle.R
    vis = (flags & oracle.F_VISIBLE) != 0
    gvis = sp["rect"][..., 0] <= sp["rect"][..., 1]
    assert np.array_equal(vis, gvis)
    np.testing.assert_array_equal(sp["rect"][vis], rect[vis])
    # tile counts
    tx = (rect[..., 1] // 16 - rect[..., 0] // 16 + 1) * (rect[..., 3] // 16 - rect[..., 2] // 16 + 1)
    np.testing.assert_array_equal(tt[vis], tx[vis])
    assert (tt[~vis] == 0).all()
    # the binning records: depth bits, first and last tile column and row,
    # tile count; zero for culled splats
    np.testing.assert_array_equal(br, _pack_bin_records(rect, sp["z"], (16, 16)))
    g, o = sp[vis], rec[vis]

    def rel(got, ref, what, tol=1e-5):
        got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
        scale = np.abs(ref).max(axis=0, keepdims=True) if ref.ndim > 1 else np.abs(ref).max()
        err = np.abs(got - ref) / (np.abs(ref) + 1e-3 * scale)
        assert err.max() <= tol, (what, err.max())

    np.testing.assert_allclose(g["uc"], o[:, R["uc"]], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(g["vc"], o[:, R["vc"]], rtol=1e-12, atol=1e-9)
    assert np.array_equal(g["z"], o[:, R["z"]].astype(np.float32))  # same FP64 value, one rounding
    rel(g["opacity"], o[:, R["o"]], "opacity", 1e-7)
    rel(g["rgb"], o[:, [R["r"], R["g"], R["bl"]]], "rgb")
    rel(g["p"], o[:, [R["p0"], R["p1"]]], "p")
    rel(g["n"], o[:, [R["n0"], R["n1"], R["n2"]]], "n")
    # conic implied by the factored form: 2/log2(e) (w01 w01^T + w23 w23^T)
    w = g["w"].astype(np.float64)
    k = 2.0 / np.log2(np.e)
    a = k * (w[:, 0] ** 2 + w[:, 2] ** 2)
    b = k * (w[:, 0] * w[:, 1] + w[:, 2] * w[:, 3])
    c = k * (w[:, 1] ** 2 + w[:, 3] ** 2)
    conic = o[:, [R["a"], R["b"], R["c"]]]
    scale = np.maximum(np.abs(conic[:, 0]), np.abs(conic[:, 2]))
    for got, j in ((a, 0), (b, 1), (c, 2)):
        err = np.abs(got - conic[:, j]) / scale
        assert err.max() < 1e-6, ("conic", j, err.max())


# ---------------------------------------------------------------------------
# binning / sorting

def _pack_bin_records(rect, z, tile):
    """rade_project's 16-byte binning records for pixel rects (x0, x1, y0,
    y1; empty when x0 > x1) and float32 depths: (bits of z, tx0 | ty0 << 16,
    tx1 | ty1 << 16, tile count), zero for an empty rect."""
    rect = np.asarray(rect, np.int64)
    vis = rect[..., 0] <= rect[..., 1]
    tx0, tx1 = rect[..., 0] // tile[0], rect[..., 1] // tile[0]
    ty0, ty1 = rect[..., 2] // tile[1], rect[..., 3] // tile[1]
    out = np.zeros(rect.shape[:-1] + (4,), np.uint32)
    out[..., 0] = np.ascontiguousarray(z, np.float32).view(np.uint32)
    out[..., 1] = tx0 | (ty0 << 16)
    out[..., 2] = tx1 | (ty1 << 16)
    out[..., 3] = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
    out[~vis] = 0
    return out


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (16, 32), (32, 16)])
def test_bin_sort_bit_exact_on_shared_input(tile):
    # Both sides fed the same rects and depths: the oracle's projection of a
    # 2-view orbit scene (so depths tie and views differ).
    import torch
    from paper_2406_01467_amd import _lib
    dev = device()
    scene = synth.make_scene_clusters(20000, seed=5, width=320, height=200)
    views = [synth.identity_view(320, 200),
             synth.make_views_orbit(scene.means.mean(0), 12.0, 1, seed=6, sizes=[(257, 190)])[0]]
    s = _settings(tile_w=tile[0], tile_h=tile[1], sh_degree=3)
    rec, rect, flags = oracle.project(oracle_settings(s), views, scene)
    z = rec[..., oracle.R["z"]].astype(np.float32)
    z[0, :300] = z[0, 300]  # ties resolved by id
    ids_ref, keys_ref, ranges_ref = oracle.bin_pairs(views, rect, z, tile)
    say("bin exact", tile, len(ids_ref))
    br = _pack_bin_records(rect, z, tile)
    vis = rect[..., 0] <= rect[..., 1]
    tt = np.where(vis, (rect[..., 1] // tile[0] - rect[..., 0] // tile[0] + 1) *
                  (rect[..., 3] // tile[1] - rect[..., 2] // tile[1] + 1), 0).astype(np.int32)
    vc = _lib.make_views(views)
    P, T = _lib.rade_views_prepare(s, vc)
    vdev = _lib.views_to_device(vc, dev)
    br_d = torch.from_numpy(br.view(np.int32).reshape(-1).copy()).to(dev)
    tt_d = torch.from_numpy(tt.reshape(-1)).to(dev)
    cap = len(ids_ref) + 37
    ids = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    keys = torch.zeros(cap, dtype=torch.int64, device=dev)
    ranges = torch.empty(2 * T, dtype=torch.int32, device=dev)
    ndev = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(_lib.rade_bin_sort_workspace(2, scene.n, cap, T), dtype=torch.uint8, device=dev)
    code, M = _lib.rade_bin_sort(s, vc, vdev, 2, scene.n, tt_d, br_d, ids, ranges, keys, cap, ndev, ws)
    torch.cuda.synchronize()
    assert code == 0 and M == len(ids_ref) and int(ndev.item()) == M
    assert np.array_equal(ids[:M].cpu().numpy().view(np.uint32), ids_ref)
    assert np.array_equal(keys[:M].cpu().numpy().view(np.uint64), keys_ref)
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), ranges_ref)
    assert (ids[M:].cpu().numpy() == -7).all()  # nothing written past M


@pytest.mark.parametrize("sizes", [[(2400, 1800)], [(2400, 1800), (2304, 1900)]])
def test_bin_sort_nine_bit_tile_digits(sizes):
    # 67,500 and 135,900 tiles of 8x8 pixels: 17- and 18-bit tile keys,
    # sorted in two 9-bit passes (the emission counts 9-bit digits)
    import torch
    from paper_2406_01467_amd import _lib
    dev = device()
    tile = (8, 8)
    scene = synth.make_scene_clusters(30000, seed=9, width=sizes[0][0], height=sizes[0][1])
    views = [synth.identity_view(*sizes[0])]
    if len(sizes) > 1:
        views.append(synth.make_views_orbit(scene.means.mean(0), 12.0, 1, seed=10,
                                            sizes=[sizes[1]])[0])
    s = _settings(tile_w=tile[0], tile_h=tile[1], sh_degree=3)
    rec, rect, flags = oracle.project(oracle_settings(s), views, scene)
    z = rec[..., oracle.R["z"]].astype(np.float32)
    ids_ref, keys_ref, ranges_ref = oracle.bin_pairs(views, rect, z, tile)
    br = _pack_bin_records(rect, z, tile)
    vis = rect[..., 0] <= rect[..., 1]
    tt = np.where(vis, (rect[..., 1] // tile[0] - rect[..., 0] // tile[0] + 1) *
                  (rect[..., 3] // tile[1] - rect[..., 2] // tile[1] + 1), 0).astype(np.int32)
    vc = _lib.make_views(views)
    P, T = _lib.rade_views_prepare(s, vc)
    assert T > 65536
    say("bin 9-bit", sizes, T, len(ids_ref))
    vdev = _lib.views_to_device(vc, dev)
    V = len(views)
    br_d = torch.from_numpy(br.view(np.int32).reshape(-1).copy()).to(dev)
    tt_d = torch.from_numpy(tt.reshape(-1)).to(dev)
    cap = len(ids_ref) + 5
    ids = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    keys = torch.zeros(cap, dtype=torch.int64, device=dev)
    ranges = torch.empty(2 * T, dtype=torch.int32, device=dev)
    ndev = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(_lib.rade_bin_sort_workspace(V, scene.n, cap, T), dtype=torch.uint8, device=dev)
    code, M = _lib.rade_bin_sort(s, vc, vdev, V, scene.n, tt_d, br_d, ids, ranges, keys, cap, ndev, ws)
    torch.cuda.synchronize()
    assert code == 0 and M == len(ids_ref) and int(ndev.item()) == M
    assert np.array_equal(ids[:M].cpu().numpy().view(np.uint32), ids_ref)
    assert np.array_equal(keys[:M].cpu().numpy().view(np.uint64), keys_ref)
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), ranges_ref)
    assert (ids[M:].cpu().numpy() == -7).all()


@pytest.mark.parametrize("name,n,tile", [("plain_64x64_1k", None, (16, 16)),
                                         ("plain_800x800_200k", 20000, (16, 16)),
                                         ("plain_800x800_200k", 20000, (8, 8)),
                                         ("plain_1600x1064_1m", None, (16, 16))])
def test_bin_sort_end_to_end(name, n, tile):
    import torch
    dev = device()
    scene, views = _workload(name, n)
    s = _settings(sh_degree=scene.sh_degree, tile_w=tile[0], tile_h=tile[1])
    sp, tt, rast, _ = _gpu_splats(scene, views, s, dev)
    rec, rect, flags = oracle.project(oracle_settings(s), views, scene)
    ids_ref, keys_ref, ranges_ref = oracle.bin_pairs(views, rect, rec[..., oracle.R["z"]].astype(np.float32), tile)
    params = to_dev(scene, dev)
    splats, ttd, brec = rast.project(*params)
    pair_ids, ranges, M, keys = rast.bin_sort(scene.n, ttd, brec, want_keys=True)
    torch.cuda.synchronize()
    say("bin e2e", name, tile, M)
    assert M == len(ids_ref)
    assert np.array_equal(pair_ids.cpu().numpy().view(np.uint32), ids_ref)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), keys_ref)
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), ranges_ref)


def test_capacity_overflow_reports_and_retries():
    import torch
    from paper_2406_01467_amd import _lib
    dev = device()
    scene, views = _workload("plain_64x64_1k")
    s = _settings()
    from paper_2406_01467_amd.raster import Rasterizer
    rast = Rasterizer(views, s, dev)
    splats, tt, brec = rast.project(*to_dev(scene, dev))
    cap = 10
    ids = torch.full((cap,), -3, dtype=torch.int32, device=dev)
    ranges = torch.full((2 * rast.total_tiles,), 5, dtype=torch.int32, device=dev)
    ndev = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(_lib.rade_bin_sort_workspace(1, scene.n, cap, rast.total_tiles), dtype=torch.uint8, device=dev)
    code, M = _lib.rade_bin_sort(s, rast.views_c, rast.views_dev, 1, scene.n, tt, brec, ids, ranges, None, cap, ndev, ws)
    torch.cuda.synchronize()
    assert code == _lib.RADE_ERR_CAPACITY and M > cap and int(ndev.item()) == M
    assert (ranges.cpu().numpy() == 0).all() and (ids.cpu().numpy() == -3).all()
    # asynchronous form (no host count): flag in n_pairs, empty ranges
    ranges.fill_(5)
    code, _ = _lib.rade_bin_sort(s, rast.views_c, rast.views_dev, 1, scene.n, tt, brec, ids, ranges, None, cap, ndev, ws, sync_count=False)
    torch.cuda.synchronize()
    assert code == 0 and int(ndev.item()) == M and (ranges.cpu().numpy() == 0).all()
    # retry with enough capacity succeeds
    ids2 = torch.empty(M, dtype=torch.int32, device=dev)
    ws2 = torch.empty(_lib.rade_bin_sort_workspace(1, scene.n, M, rast.total_tiles), dtype=torch.uint8, device=dev)
    code, M2 = _lib.rade_bin_sort(s, rast.views_c, rast.views_dev, 1, scene.n, tt, brec, ids2, ranges, None, M, ndev, ws2)
    assert code == 0 and M2 == M


# ---------------------------------------------------------------------------
# forward maps

def _full_parity(scene, views, s, label):
    dev = device()
    rast, maps, gv, _ = gpu_forward(scene, views, s, dev)
    st = oracle_settings(s)
    rec, rect, flags, outs = oracle.forward(st, views, scene)
    nfrag = 0
    for vi in range(len(views)):
        nfrag += compare_maps(gv[vi], outs[vi], label=f"{label} view {vi}: ")
    tot = sum(v.pixels for v in views)
    say(label, "fragile pixels", nfrag, "of", tot, "mean blends",
        float(np.mean([o["count"].mean() for o in outs])))
    assert nfrag <= max(2, 1e-2 * tot)
    return gv, outs


def test_render_fwd_64x64_full():
    scene, views = _workload("plain_64x64_1k")
    _full_parity(scene, views, _settings(), "64x64")


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 16), (16, 32), (16, 8), (8, 16)])
def test_render_fwd_ragged_tiles(tile):
    # image size not a multiple of any tile size; several tiles; SH degree 3
    scene = synth.make_scene_ball(6000, seed=11, centre=(0.0, 0.0, 3.0), radius=1.2,
                                  log_scale_mu=-3.2)
    views = [synth.identity_view(100, 70)]
    _full_parity(scene, views, _settings(tile_w=tile[0], tile_h=tile[1], sh_degree=3),
                 f"ragged {tile}")


def test_render_fwd_two_uneven_views_with_background():
    scene = synth.make_scene_clusters(8000, seed=7, width=120, height=90, dist_range=(2, 6))
    views = [synth.identity_view(120, 90)] + synth.make_views_orbit(
        scene.means.mean(0), 5.0, 1, seed=8, sizes=[(77, 131)])
    _full_parity(scene, views, _settings(sh_degree=3, bg=(0.25, 0.5, 1.0)), "2 views")


def _sampled_parity(name, npix, seed, tile=(16, 16), schedule=0):
    dev = device()
    scene, views = _workload(name)
    s = _settings(sh_degree=scene.sh_degree, tile_w=tile[0], tile_h=tile[1], schedule=schedule)
    say("sampled parity", name, "N", scene.n, "pixels", npix)
    rast, maps, gv, _ = gpu_forward(scene, views, s, dev)
    v = views[0]
    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(v.pixels, npix, replace=False)).astype(np.int64)
    st = oracle_settings(s)
    rec, rect, flags = oracle.project(st, views, scene)
    out = oracle.render(st, v, rec[0], flags[0], pix)
    nfrag = compare_maps(gv[0], out, pixels=pix, label=name + ": ")
    say(name, "fragile", nfrag, "mean blends", out["count"].mean())
    assert nfrag <= max(2, 0.01 * npix)
    return gv, out, pix


def test_render_fwd_800x800_200k_sampled():
    _sampled_parity("plain_800x800_200k", 600, 21)


def test_render_fwd_1600x1064_1m_sampled():
    # the benchmark's workload in its launch configuration (16x16 tiles,
    # heavy-first order), 16,384 seeded pixels
    _sampled_parity("plain_1600x1064_1m", 16384, 22, schedule=1)


def test_tile_size_invariance():
    # Every map is bitwise identical across the six tile sizes: each pixel
    # blends the same splats in the same order with the same FP32 operations
    # (splat centres are rounded relative to a 32-pixel-aligned origin that
    # depends on the pixel only).  The image is 100x70 so the last tiles are
    # ragged for every size; the scene puts splats across tile borders.
    dev = device()
    scene = synth.make_scene_ball(5000, seed=12, centre=(0.0, 0.0, 3.0), radius=1.0, log_scale_mu=-3.0)
    views = [synth.identity_view(100, 70)]
    res = {}
    for tile in [(8, 8), (16, 16), (32, 16), (16, 32), (16, 8), (8, 16)]:
        _, _, gv, _ = gpu_forward(scene, views, _settings(tile_w=tile[0], tile_h=tile[1], sh_degree=3), dev)
        res[tile] = gv[0]
    base = res[(16, 16)]
    assert base["count"].sum() > 100000
    for tile, g in res.items():
        for k in ("count", "median", "last_id", "color", "depth", "normal", "alpha", "t_final"):
            a, b = np.asarray(g[k]), np.asarray(base[k])
            nbad = int((a.view(np.uint32) != b.view(np.uint32)).sum()) if a.dtype == np.float32 \
                else int((a != b).sum())
            say(f"tile {tile} {k}: {nbad} pixels differ from 16x16")
            assert nbad == 0, (tile, k, nbad)


def _needle_scene(n, seed):
    # strongly anisotropic Gaussians (one long axis, two thin ones) at random
    # orientations: their support boxes are far larger than the pixels they
    # reach, which is what the 8x8 tiles' per-row lane masks cut away
    scene = synth.make_scene_ball(n, seed=seed, centre=(0.0, 0.0, 3.0), radius=1.0,
                                  log_scale_mu=-4.0, log_scale_sd=0.3)
    rng = np.random.default_rng(seed + 100)
    long_axis = rng.integers(0, 3, n)
    scene.scales[np.arange(n), long_axis] *= np.float32(15.0)
    return scene


def test_lane_masks_keep_every_blend_of_needle_splats():
    # 8x8 tiles (one wave per tile, lane masks from per-row ellipse
    # intervals) against 16x16 tiles (no lane masks): bitwise equal maps and
    # saved state, gradients equal up to the order of the FP32 atomics; and
    # the 8x8 maps and gradients against the oracle
    import torch
    dev = device()
    from paper_2406_01467_amd.raster import Rasterizer
    scene = _needle_scene(6000, 41)
    views = [synth.identity_view(100, 70)]
    params = to_dev(scene, dev)
    outs = {}
    for tile, lm in ((16, 0), (8, 0), (16, 1)):
        s = _settings(sh_degree=3, tile_w=tile, tile_h=tile, schedule=1, lane_masks=lm)
        rast = Rasterizer(views, s, dev)
        # (the counting pass exists for the default shapes only)
        maps = rast.forward(*params, want_count=lm == 0)
        rng = np.random.default_rng(4)
        P = rast.total_pixels
        g = [torch.from_numpy(rng.normal(size=k * P).astype(np.float32)).to(dev) for k in (3, 2, 3, 1)]
        grads = rast.backward(maps.state, *params, *g)
        torch.cuda.synchronize()
        outs[(tile, lm)] = (maps, [x.cpu().numpy() for x in grads])
    m0, g0 = outs[(16, 0)]
    assert int(m0.count.sum()) > 50000
    for key in ((8, 0), (16, 1)):
        m1, g1 = outs[key]
        keys = ("color", "depth", "normal", "alpha") + (("count",) if m1.count is not None else ())
        for k in keys:
            assert torch.equal(getattr(m0, k), getattr(m1, k)), (key, k)
        for k in ("t_final", "median"):
            assert torch.equal(getattr(m0.state, k), getattr(m1.state, k)), (key, k)
        for a, b in zip(g0, g1):
            say(f"  {key} vs 16x16 gradient difference, normwise: "
                f"{np.linalg.norm(a - b) / np.linalg.norm(a):.3g}")
    # the gradients of both tile sizes against the oracle's adjoint (their
    # atomics sum each Gaussian's pixels in different groups, and the long
    # splats' gradients cancel heavily, so they are compared with the oracle
    # rather than with each other)
    s8 = _settings(sh_degree=3, tile_w=8, tile_h=8, schedule=1)
    _full_parity(scene, views, s8, "needles 8x8")
    _bwd_parity(scene, views, s8, 42, "bwd needles 8x8")
    # four 64-splat chunks per staging round in the quadrant backward
    _bwd_parity(scene, views, _settings(sh_degree=3, tile_w=8, tile_h=8, schedule=1, batch=256),
                43, "bwd needles 8x8 batch 256")
    _bwd_parity(scene, views, _settings(sh_degree=3, schedule=1), 42, "bwd needles 16x16")
    # 16x16 tiles with lane masks on each of the four waves
    _bwd_parity(scene, views, _settings(sh_degree=3, schedule=1, lane_masks=1), 44,
                "bwd needles 16x16 lane masks")


def test_degenerate_inputs():
    # no Gaussian, all culled (behind camera, NaN, tiny opacity), zero quaternion
    import torch
    dev = device()
    from paper_2406_01467_amd.raster import Rasterizer
    v = [synth.identity_view(40, 24)]
    s = _settings()
    for sc in (scene_from(np.zeros((0, 3)), np.zeros((0, 3))),
               scene_from([[0, 0, -1.0], [np.nan, 0, 3], [0, 0, 3], [0, 0, 0.1]],
                          [[0.1] * 3] * 4, opac=[0.5, 0.5, 0.001, 0.5])):
        rast = Rasterizer(v, _settings(bg=(0.1, 0.2, 0.3)), dev)
        maps = rast.forward(*to_dev(sc, dev), want_count=True)
        torch.cuda.synchronize()
        assert maps.state.n_pairs == 0
        c = maps.color.cpu().numpy().reshape(3, -1)
        np.testing.assert_allclose(c, np.array([0.1, 0.2, 0.3], np.float32)[:, None] * np.ones((3, 960)))
        assert (maps.alpha.cpu().numpy() == 0).all() and (maps.state.t_final.cpu().numpy() == 1).all()
        assert (maps.state.median.cpu().numpy() == -1).all() and (maps.count.cpu().numpy() == 0).all()
    # one Gaussian covering everything with opacity 1: alpha clamps at 0.99
    # near its centre, never exceeds it, and equals o exp(-power) elsewhere
    sc = scene_from([[0, 0, 2.0]], [[5.0] * 3], opac=[1.0], rgb=[[1, 0, 0]])
    rast = Rasterizer(v, s, dev)
    maps = rast.forward(*to_dev(sc, dev))
    a = maps.alpha.cpu().numpy().reshape(24, 40)
    assert a.max() <= np.float32(0.99) and a[12, 20] == np.float32(0.99)
    st = oracle_settings(s)
    rec, rect, flags, outs = oracle.forward(st, v, sc)
    np.testing.assert_allclose(a.reshape(-1), outs[0]["alpha"], rtol=1e-5)


# ---------------------------------------------------------------------------
# backward

def _bwd_parity(scene, views, s, seed, label, pixels=None, recompute=False):
    import torch
    dev = device()
    rast, maps, gv, params = gpu_forward(scene, views, s, dev, keep=not recompute)
    rng = np.random.default_rng(seed)
    P = rast.total_pixels
    gC = rng.normal(size=3 * P).astype(np.float32)
    gD = rng.normal(size=2 * P).astype(np.float32)
    gN = rng.normal(size=3 * P).astype(np.float32)
    gA = rng.normal(size=P).astype(np.float32)
    if pixels is not None:  # only sampled pixels carry upstream gradient
        mask = np.zeros(P, bool)
        mask[pixels] = True
        gC *= np.tile(mask, 3); gD *= np.tile(mask, 2); gN *= np.tile(mask, 3); gA *= mask
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    dm, ds, dq, do, dsh = rast.backward(maps.state, *params, t(gC), t(gD), t(gN), t(gA))
    torch.cuda.synchronize()
    st = oracle_settings(s)
    gouts, pix_lists = [], []
    for vi, v in enumerate(views):
        o = rast.views_c[vi].pix_offset
        Pv = v.pixels
        g = np.zeros((Pv, 9))
        g[:, 0:3] = gC[3 * o: 3 * o + 3 * Pv].reshape(3, Pv).T
        g[:, 3:5] = gD[2 * o: 2 * o + 2 * Pv].reshape(2, Pv).T
        g[:, 5:8] = gN[3 * o: 3 * o + 3 * Pv].reshape(3, Pv).T
        g[:, 8] = gA[o: o + Pv]
        if pixels is not None:
            pl = pixels[(pixels >= o) & (pixels < o + Pv)] - o
            pix_lists.append(pl.astype(np.int64))
            gouts.append(g[pl])
        else:
            gouts.append(g)
    pl = pix_lists if pixels is not None else None
    ref = oracle.backward(st, views, scene, gouts, pixels=pl)
    scale = oracle.gradient_error_scale(st, views, scene, gouts, pixels=pl)
    got = dict(means=dm.cpu().numpy(), scales=ds.cpu().numpy(), quats=dq.cpu().numpy(),
               opacities=do.cpu().numpy(), sh=dsh.cpu().numpy())
    grad_check(got, ref, scale, label)


def test_render_bwd_64x64_full():
    scene, views = _workload("plain_64x64_1k")
    _bwd_parity(scene, views, _settings(), 31, "bwd 64x64")


def test_render_bwd_two_views_sh3():
    scene = synth.make_scene_clusters(3000, seed=9, width=80, height=64, dist_range=(2, 5))
    views = [synth.identity_view(80, 64)] + synth.make_views_orbit(
        scene.means.mean(0), 4.0, 1, seed=10, sizes=[(70, 50)])
    _bwd_parity(scene, views, _settings(sh_degree=3, bg=(0.3, 0.1, 0.2)), 32, "bwd 2 views")


def test_render_bwd_recompute_mode():
    scene = synth.make_scene_ball(4000, seed=13, centre=(0.0, 0.0, 3.0), radius=1.0, log_scale_mu=-3.0)
    views = [synth.identity_view(64, 48)]
    _bwd_parity(scene, views, _settings(sh_degree=3), 33, "bwd recompute", recompute=True)


def test_render_bwd_800x800_200k_sampled_pixels():
    scene, views = _workload("plain_800x800_200k")
    rng = np.random.default_rng(34)
    pix = np.sort(rng.choice(views[0].pixels, 1024, replace=False)).astype(np.int64)
    _bwd_parity(scene, views, _settings(sh_degree=3), 35, "bwd 800x800 sampled", pixels=pix)


def test_render_bwd_1600x1064_1m_sampled_pixels():
    # The benchmark's workload (1M Gaussians, one 1600x1064 view, SH degree
    # 3) in its launch configuration (16x16 tiles, heavy-first order): the
    # VJP of 2,048 seeded pixels against the oracle's adjoint, over every
    # Gaussian.
    scene, views = _workload("plain_1600x1064_1m")
    rng = np.random.default_rng(36)
    pix = np.sort(rng.choice(views[0].pixels, 2048, replace=False)).astype(np.int64)
    _bwd_parity(scene, views, _settings(sh_degree=3, schedule=1), 37, "bwd 1600x1064 sampled",
                pixels=pix)


def test_alpha_min_setting_fwd_bwd():
    # a non-default alpha_min (1e-3 instead of 1/255): the support rects,
    # the cull and the per-pixel skip all follow it; maps and gradients
    # against the oracle run with the same setting
    scene = synth.make_scene_ball(6000, seed=16, centre=(0.0, 0.0, 3.0), radius=1.2,
                                  log_scale_mu=-3.2)
    scene.opacities[:300] = np.float32(2e-3)  # between 1e-3 and 1/255: kept now
    views = [synth.identity_view(100, 70)]
    s = _settings(sh_degree=3, alpha_min=1e-3)
    _full_parity(scene, views, s, "alpha_min 1e-3")
    _bwd_parity(scene, views, s, 38, "bwd alpha_min 1e-3")


@pytest.mark.parametrize("schedule", [1, 2])
def test_schedules_match_one_workgroup_per_tile(schedule):
    # Heavy-first order and the persistent work queue change only which
    # workgroup processes a tile: maps are bitwise identical, gradients equal
    # up to the order of the FP32 atomic additions.
    import torch
    dev = device()
    from paper_2406_01467_amd.raster import Rasterizer
    scene = synth.make_scene_clusters(20000, seed=14, width=200, height=150, dist_range=(2, 8))
    views = [synth.identity_view(200, 150)] + synth.make_views_orbit(
        scene.means.mean(0), 8.0, 2, seed=15, sizes=[(170, 96), (64, 200)])
    params = to_dev(scene, dev)
    outs = {}
    for sch in (0, schedule):
        rast = Rasterizer(views, _settings(sh_degree=3, schedule=sch), dev)
        maps = rast.forward(*params, want_count=True)
        rng = np.random.default_rng(3)
        P = rast.total_pixels
        g = [torch.from_numpy(rng.normal(size=k * P).astype(np.float32)).to(dev) for k in (3, 2, 3, 1)]
        grads = rast.backward(maps.state, *params, *g)
        torch.cuda.synchronize()
        outs[sch] = (maps, [x.cpu().numpy() for x in grads])
    m0, g0 = outs[0]
    m1, g1 = outs[schedule]
    for k in ("color", "depth", "normal", "alpha", "count"):
        assert torch.equal(getattr(m0, k), getattr(m1, k)), k
    for k in ("t_final", "last", "median"):
        assert torch.equal(getattr(m0.state, k), getattr(m1.state, k)), k
    for a, b in zip(g0, g1):
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a)
