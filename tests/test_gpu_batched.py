"""Batched multi-view path: one key space over uneven views, HIP-graph replay,
tile order, capacity overflow handling and the autotuner."""
import numpy as np
import pytest

import synth
from gpu_common import device, say, to_dev

pytestmark = pytest.mark.gpu


def _scene_views(n=20000, seed=21):
    scene = synth.make_scene_clusters(n, seed=seed, width=240, height=160, dist_range=(2, 8))
    views = synth.make_views_orbit(scene.means.mean(0), 7.0, 4, seed=seed + 1,
                                   size_range=((60, 240), (40, 180)))
    return scene, views


def _fixed_grads(P, dev, seed=5):
    import torch
    rng = np.random.default_rng(seed)
    return [torch.from_numpy(rng.normal(size=k * P).astype(np.float32)).to(dev) for k in (3, 2, 3, 1)]


@pytest.mark.parametrize("schedule,tile,lm", [(0, (16, 16), 0), (1, (8, 8), 0), (2, (16, 16), 0),
                                              (2, (32, 16), 0), (1, (16, 16), 1), (2, (16, 16), 1),
                                              (0, (32, 16), 1)])
def test_graph_replay_equals_plain_path(schedule, tile, lm):
    """Replays of the captured step equal the plain path's maps bit for bit
    and its gradients to FP32 atomic order; with lane masks (lm) both paths
    also pass the forward's mask cache to the backward."""
    import torch
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene_views()
    st = Settings(tile_w=tile[0], tile_h=tile[1], sh_degree=3, schedule=schedule, lane_masks=lm)
    params = to_dev(scene, dev)
    rast = Rasterizer(views, Settings(tile_w=tile[0], tile_h=tile[1], sh_degree=3, lane_masks=lm),
                      dev)
    g = _fixed_grads(rast.total_pixels, dev)
    ref = rast.forward(*params, want_count=False)
    ref_grads = [x.clone() for x in rast.backward(ref.state, *params, *g)]
    plan = BatchedPlan(views, st, params, lambda maps: g)
    assert (plan.lane_masks is not None) == (lm == 1 or tile == (8, 8))
    plan.capture()
    for rep in range(3):
        plan.replay()
        # eager work between replays (the plain path again)
        other = rast.forward(*params)
        torch.cuda.synchronize()
        assert not plan.overflowed()
        for k in ("color", "depth", "normal", "alpha", "t_final", "last", "median"):
            want = getattr(ref, k) if hasattr(ref, k) else getattr(ref.state, k)
            assert torch.equal(plan.maps[k], want), (rep, k)
        for a, b in zip(plan.grads, ref_grads):
            assert torch.linalg.norm(a - b) <= 1e-6 * torch.linalg.norm(b), rep
        del other
    say("graph replay ok", schedule, tile, "pairs", plan.n_pairs())


@pytest.mark.parametrize("lm", [0, 1])
def test_capacity_overflow_grows_and_recaptures(lm):
    """A plan sized for 100 pairs overflows, grows (with lane masks, also the
    forward's mask cache) and re-captures: the second replay equals the
    plain path."""
    import torch
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene_views(8000, seed=31)
    params = to_dev(scene, dev)
    st = Settings(sh_degree=3, schedule=2, lane_masks=lm)
    rast = Rasterizer(views, Settings(sh_degree=3, lane_masks=lm), dev)
    g = _fixed_grads(rast.total_pixels, dev)
    ref = rast.forward(*params)
    ref_grads = [x.clone() for x in rast.backward(ref.state, *params, *g)]
    plan = BatchedPlan(views, st, params, lambda maps: g, capacity=100)
    n = plan.step()
    torch.cuda.synchronize()
    assert n == 2 and plan.capacity >= plan.n_pairs() and plan.n_pairs() == ref.state.n_pairs
    assert torch.equal(plan.maps["color"], ref.color)
    if lm:
        assert plan.lane_masks is not None
        assert plan.lane_masks.numel() * 8 >= plan.capacity * 4 * 8
    for a, b in zip(plan.grads, ref_grads):
        assert torch.linalg.norm(a - b) <= 1e-6 * torch.linalg.norm(b)


@pytest.mark.parametrize("large", [False, True])
def test_tile_order_is_heavy_first_permutation(large):
    # small: one workgroup sorts all tiles; large (more than 16384 tiles of
    # 8x8 pixels): the radix pass over a key array
    import torch
    from paper_2406_01467_amd import Settings, _lib
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene_views(10000, seed=41)
    st = Settings(sh_degree=3, schedule=1)
    if large:
        views = [synth.identity_view(1200, 900)]
        st = Settings(sh_degree=3, schedule=1, tile_w=8, tile_h=8)
    rast = Rasterizer(views, st, dev)
    assert (rast.total_tiles > 16384) == large
    splats, tt, brec = rast.project(*to_dev(scene, dev))
    _, ranges, M = rast.bin_sort(scene.n, tt, brec)
    order = rast.tile_order(ranges)
    torch.cuda.synchronize()
    o = order.cpu().numpy()[:-1].astype(np.int64)
    r = ranges.cpu().numpy().reshape(-1, 2).astype(np.int64)
    assert np.array_equal(np.sort(o), np.arange(rast.total_tiles))
    lens = (r[:, 1] - r[:, 0])[o]
    bucket = np.where(lens == 0, 0, np.minimum(255, np.floor(16 * np.log2(lens + 1.0))))
    assert np.all(np.diff(bucket) <= 0)
    # stable within a bucket: ascending tile index
    same = np.diff(bucket) == 0
    assert np.all(np.diff(o)[same] > 0)


def test_autotuner_picks_a_candidate_and_caches(tmp_path, monkeypatch):
    import torch
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import autotune
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    monkeypatch.setenv("RADE_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    scene, views = _scene_views(8000, seed=51)
    params = to_dev(scene, dev)
    P = Rasterizer(views, Settings(), dev).total_pixels
    g = _fixed_grads(P, dev)
    best, timings = autotune(views, params, Settings(sh_degree=3), lambda m: g,
                             tiles=[(8, 8), (16, 16)], schedules=[0, 2], reps=2)
    # stage 1: every (tile, schedule), and with lane masks on the tiles of
    # several 8x8 waves; stage 2: wave shapes x batches of the best plain one
    stage1 = {k: v for k, v in timings.items() if "/w" not in k}
    assert sorted(stage1) == ["16x16/0", "16x16/0/lm", "16x16/2", "16x16/2/lm", "8x8/0", "8x8/2"]
    b1 = min((k for k in stage1 if not k.endswith("/lm")), key=stage1.get)
    stage2 = [k for k in timings if "/w" in k]
    assert stage2 and all(k.startswith(b1 + "/w") for k in stage2)
    key = f"{best.tile_w}x{best.tile_h}/{best.schedule}"
    if best.wave_w or best.batch:
        key += f"/w{best.wave_w}/b{best.batch}"
    if best.lane_masks:
        key += "/lm"
    assert key in timings and timings[key] == min(timings.values())
    again, t2 = autotune(views, params, Settings(sh_degree=3), lambda m: g,
                         tiles=[(8, 8), (16, 16)], schedules=[0, 2], reps=2)
    assert (again.tile_w, again.tile_h, again.schedule, again.wave_w, again.batch,
            again.lane_masks) == \
        (best.tile_w, best.tile_h, best.schedule, best.wave_w, best.batch, best.lane_masks)
    say("autotune", timings)


def test_batched_16views_1m_against_the_oracle():
    """The 16-view workload (1M Gaussians, uneven orbit views) through the
    batched plan at its tuned launch shape (16x16 tiles with lane masks on
    their four 8x8 waves, heavy-first order), graph-replayed: maps of three views on
    sampled pixels against the oracle, and the VJP of upstream gradients on
    sampled pixels of those views (zero elsewhere) against the oracle's
    adjoint over all 1M Gaussians."""
    import torch
    import oracle
    from gpu_common import compare_maps, grad_check, oracle_settings
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan
    dev = device()
    scene, views = synth.make_workload("batched_16views_1m")
    st = Settings(tile_w=16, tile_h=16, sh_degree=3, schedule=1, lane_masks=1)
    params = to_dev(scene, dev)
    rng = np.random.default_rng(61)
    sel = [0, 7, 13]
    from paper_2406_01467_amd.raster import Rasterizer
    vc = Rasterizer(views, st, dev).views_c
    P = sum(v.pixels for v in views)
    fwd_pix = {vi: np.sort(rng.choice(views[vi].pixels, 4096, replace=False)).astype(np.int64)
               for vi in sel}
    bwd_pix = {vi: np.sort(rng.choice(views[vi].pixels, 700, replace=False)).astype(np.int64)
               for vi in sel}
    gC = np.zeros(3 * P, np.float32)
    gD = np.zeros(2 * P, np.float32)
    gN = np.zeros(3 * P, np.float32)
    gA = np.zeros(P, np.float32)
    gouts = []
    for vi in sel:
        o, Pv, pl = vc[vi].pix_offset, views[vi].pixels, bwd_pix[vi]
        g = rng.normal(size=(len(pl), 9)).astype(np.float32)
        for c in range(3):
            gC[3 * o + c * Pv + pl] = g[:, c]
            gN[3 * o + c * Pv + pl] = g[:, 5 + c]
        for c in range(2):
            gD[2 * o + c * Pv + pl] = g[:, 3 + c]
        gA[o + pl] = g[:, 8]
        gouts.append(g.astype(np.float64))
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    grads_in = [t(gC), t(gD), t(gN), t(gA)]
    say("batched 16 views: capture and replay")
    plan = BatchedPlan(views, st, params, lambda maps: grads_in)
    plan.step()
    plan.replay()
    torch.cuda.synchronize()
    assert not plan.overflowed()
    say("batched 16 views: pairs", plan.n_pairs())
    pair_ids = plan.pair_ids[: plan.n_pairs()].cpu().numpy().astype(np.int64)
    ranges = plan.ranges.cpu().numpy().astype(np.int64).reshape(-1, 2)
    s_or = oracle_settings(st)
    sub_views = [views[vi] for vi in sel]
    rec, _, flags = oracle.project(s_or, sub_views, scene)
    for k, vi in enumerate(sel):
        v, o = views[vi], vc[vi].pix_offset
        Pv, H, W = v.pixels, v.height, v.width
        d = {}
        for name, ch in (("color", 3), ("depth", 2), ("normal", 3), ("alpha", 1),
                         ("t_final", 1), ("median", 1), ("last", 1)):
            d[name] = plan.maps[name][ch * o: ch * o + ch * Pv].view(ch, H, W).cpu().numpy()
        py, px = np.mgrid[0:H, 0:W]
        tile = vc[vi].tile_offset + (py // st.tile_h) * vc[vi].tiles_x + px // st.tile_w
        last = d["last"][0]
        d["last_id"] = np.where(last >= 0, pair_ids[np.clip(ranges[tile, 0] + last, 0,
                                                            len(pair_ids) - 1)], -1)
        out = oracle.render(s_or, v, rec[k], flags[k], fwd_pix[vi])
        nfrag = compare_maps(d, out, pixels=fwd_pix[vi], label=f"batched view {vi}: ")
        say(f"batched view {vi} ({W}x{H}): fragile {nfrag}, mean blends {out['count'].mean():.1f}")
        assert nfrag <= max(2, 0.01 * len(fwd_pix[vi]))
    got = dict(means=plan.grads[0].cpu().numpy(), scales=plan.grads[1].cpu().numpy(),
               quats=plan.grads[2].cpu().numpy(), opacities=plan.grads[3].cpu().numpy(),
               sh=plan.grads[4].cpu().numpy().reshape(scene.sh.shape))
    pl = [bwd_pix[vi] for vi in sel]
    ref = oracle.backward(s_or, sub_views, scene, gouts, pixels=pl, rec=rec, flags=flags)
    scale = oracle.gradient_error_scale(s_or, sub_views, scene, gouts, pixels=pl)
    grad_check(got, ref, scale, "batched 16 views bwd")
