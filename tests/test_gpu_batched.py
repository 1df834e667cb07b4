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


@pytest.mark.parametrize("schedule,tile", [(0, (16, 16)), (1, (8, 8)), (2, (16, 16)), (2, (32, 16))])
def test_graph_replay_equals_plain_path(schedule, tile):
    import torch
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene_views()
    st = Settings(tile_w=tile[0], tile_h=tile[1], sh_degree=3, schedule=schedule)
    params = to_dev(scene, dev)
    rast = Rasterizer(views, Settings(tile_w=tile[0], tile_h=tile[1], sh_degree=3), dev)
    g = _fixed_grads(rast.total_pixels, dev)
    ref = rast.forward(*params, want_count=False)
    ref_grads = [x.clone() for x in rast.backward(ref.state, *params, *g)]
    plan = BatchedPlan(views, st, params, lambda maps: g)
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


def test_capacity_overflow_grows_and_recaptures():
    import torch
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene_views(8000, seed=31)
    params = to_dev(scene, dev)
    st = Settings(sh_degree=3, schedule=2)
    rast = Rasterizer(views, Settings(sh_degree=3), dev)
    g = _fixed_grads(rast.total_pixels, dev)
    ref = rast.forward(*params)
    plan = BatchedPlan(views, st, params, lambda maps: g, capacity=100)
    n = plan.step()
    torch.cuda.synchronize()
    assert n == 2 and plan.capacity >= plan.n_pairs() and plan.n_pairs() == ref.state.n_pairs
    assert torch.equal(plan.maps["color"], ref.color)


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
    splats, tt = rast.project(*to_dev(scene, dev))
    _, ranges, M = rast.bin_sort(scene.n, splats, tt)
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
    # stage 1: every (tile, schedule); stage 2: wave shapes x batches of the best
    stage1 = {k: v for k, v in timings.items() if "/w" not in k}
    assert len(stage1) == 4
    b1 = min(stage1, key=stage1.get)
    stage2 = [k for k in timings if "/w" in k]
    assert stage2 and all(k.startswith(b1 + "/w") for k in stage2)
    key = f"{best.tile_w}x{best.tile_h}/{best.schedule}"
    if best.wave_w or best.batch:
        key += f"/w{best.wave_w}/b{best.batch}"
    assert key in timings and timings[key] == min(timings.values())
    again, t2 = autotune(views, params, Settings(sh_degree=3), lambda m: g,
                         tiles=[(8, 8), (16, 16)], schedules=[0, 2], reps=2)
    assert (again.tile_w, again.tile_h, again.schedule, again.wave_w, again.batch) == \
        (best.tile_w, best.tile_h, best.schedule, best.wave_w, best.batch)
    say("autotune", timings)
