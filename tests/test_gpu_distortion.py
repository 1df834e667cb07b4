"""GPU parity of the depth-distortion term (Sec. 3.4, Eq. 23) with the FP64
oracle: the per-pixel map of the forward (maps bar: 1e-5 relative with a
floor of 1e-3 of the map's maximum, fragile pixels excluded) and the
gradients of its adjoint with detached weights (gradient bar of the other
backward tests)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import device, grad_check, oracle_settings, say, to_dev

pytestmark = pytest.mark.gpu


def _settings(**kw):
    from paper_2406_01467_amd import Settings
    return Settings(**kw)


def _check_map(got, ref, frag, label, mag, tol=1e-5):
    """|x - x_ref| <= tol (|x_ref| + 1e-3 max|x_ref| + 0.1 mag): mag is the
    oracle's first-order bound of the sum's change per unit relative error of
    the per-pixel depths (FP32 depths differ from FP64 ones by their rounding,
    which decides the accuracy of small distortions between close depths)."""
    keep = (frag & 1) == 0
    got = np.asarray(got, np.float64)[keep]
    ref = np.asarray(ref, np.float64)[keep]
    floor = 1e-3 * np.abs(ref).max() + 0.1 * np.asarray(mag, np.float64)[keep] + 1e-30
    err = np.abs(got - ref) / (np.abs(ref) + floor)
    i = int(np.argmax(err))
    say(f"  {label}: worst {err[i]:.3g} (ref {ref[i]:.6g} got {got[i]:.6g}, floor {floor[i]:.3g}); "
        f"{(~((frag & 1) == 0)).sum()} fragile")
    assert err.max() <= tol, (label, err.max())


def _forward(scene, views, s, dev):
    import torch
    from paper_2406_01467_amd.raster import Rasterizer
    rast = Rasterizer(views, s, dev)
    params = to_dev(scene, dev)
    maps = rast.forward(*params, want_count=True, want_distortion=True)
    torch.cuda.synchronize()
    return rast, maps, params


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_distortion_map_two_views(tile):
    dev = device()
    scene = synth.make_scene_clusters(4000, seed=41, width=96, height=72, dist_range=(2, 6))
    views = [synth.identity_view(96, 72)] + synth.make_views_orbit(
        scene.means.mean(0), 5.0, 1, seed=42, sizes=[(70, 54)])
    s = _settings(sh_degree=3, tile_w=tile[0], tile_h=tile[1])
    rast, maps, _ = _forward(scene, views, s, dev)
    rec, _, flags, outs = oracle.forward(oracle_settings(s), views, scene)
    for vi, v in enumerate(views):
        got = maps.view_planes(rast, vi)["distortion"].cpu().numpy().reshape(-1)
        assert np.isfinite(got).all()
        _check_map(got, outs[vi]["distortion"], outs[vi]["fragile"], f"view {vi} {tile}",
                   outs[vi]["distortion_mag"])


def test_distortion_map_1600x1064_1m_sampled():
    dev = device()
    scene, views = synth.make_workload("plain_1600x1064_1m")
    s = _settings(sh_degree=3)
    rast, maps, _ = _forward(scene, views, s, dev)
    rng = np.random.default_rng(43)
    pix = np.sort(rng.choice(views[0].pixels, 1500, replace=False)).astype(np.int64)
    st = oracle_settings(s)
    rec, _, flags = oracle.project(st, views, scene)
    ref = oracle.render(st, views[0], rec[0], flags[0], pix)
    got = maps.distortion.cpu().numpy()[pix]
    _check_map(got, ref["distortion"], ref["fragile"], "1600x1064 sampled", ref["distortion_mag"])


def test_distortion_off_leaves_other_maps_bitwise_equal():
    import torch
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene = synth.make_scene_clusters(5000, seed=44, width=80, height=64, dist_range=(2, 5))
    views = [synth.identity_view(80, 64)]
    s = _settings(sh_degree=3)
    params = to_dev(scene, dev)
    rast = Rasterizer(views, s, dev)
    a = rast.forward(*params, want_count=True, want_distortion=False)
    b = rast.forward(*params, want_count=True, want_distortion=True)
    torch.cuda.synchronize()
    for k in ("color", "depth", "normal", "alpha", "count"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert a.distortion is None and b.distortion is not None


def _bwd(scene, views, s, seed, label, with_others):
    import torch
    dev = device()
    rast, maps, params = _forward(scene, views, s, dev)
    rng = np.random.default_rng(seed)
    P = rast.total_pixels
    gL = rng.normal(size=P).astype(np.float32)
    ups = [rng.normal(size=k * P).astype(np.float32) if with_others else np.zeros(k * P, np.float32)
           for k in (3, 2, 3, 1)]
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    dm, ds, dq, do, dsh = rast.backward(maps.state, *params, *(t(u) for u in ups),
                                        d_distortion=t(gL))
    torch.cuda.synchronize()
    gC, gD, gN, gA = ups
    gouts = []
    for vi, v in enumerate(views):
        o, Pv = rast.views_c[vi].pix_offset, v.pixels
        g = np.zeros((Pv, 10))
        g[:, 0:3] = gC[3 * o: 3 * o + 3 * Pv].reshape(3, Pv).T
        g[:, 3:5] = gD[2 * o: 2 * o + 2 * Pv].reshape(2, Pv).T
        g[:, 5:8] = gN[3 * o: 3 * o + 3 * Pv].reshape(3, Pv).T
        g[:, 8] = gA[o: o + Pv]
        g[:, 9] = gL[o: o + Pv]
        gouts.append(g)
    st = oracle_settings(s)
    ref = oracle.backward(st, views, scene, gouts)
    scale = oracle.gradient_error_scale(st, views, scene, gouts)
    got = dict(means=dm.cpu().numpy(), scales=ds.cpu().numpy(), quats=dq.cpu().numpy(),
               opacities=do.cpu().numpy(), sh=dsh.cpu().numpy())
    grad_check(got, ref, scale, label)


def test_distortion_gradient_alone():
    scene = synth.make_scene_clusters(3000, seed=45, width=80, height=64, dist_range=(2, 5))
    views = [synth.identity_view(80, 64)]
    _bwd(scene, views, _settings(sh_degree=3), 46, "distortion only", with_others=False)


def test_distortion_gradient_with_all_maps_two_views():
    scene = synth.make_scene_clusters(3000, seed=47, width=80, height=64, dist_range=(2, 5))
    views = [synth.identity_view(80, 64)] + synth.make_views_orbit(
        scene.means.mean(0), 4.0, 1, seed=48, sizes=[(64, 56)])
    _bwd(scene, views, _settings(sh_degree=3, bg=(0.2, 0.1, 0.3)), 49, "all maps + distortion",
         with_others=True)


def test_autograd_distortion_output():
    import torch
    from paper_2406_01467_amd.raster import Rasterizer, render
    dev = device()
    scene = synth.make_scene_clusters(2000, seed=50, width=64, height=48, dist_range=(2, 5))
    views = [synth.identity_view(64, 48)]
    s = _settings(sh_degree=3)
    rast = Rasterizer(views, s, dev)
    leaves = [p.detach().clone().requires_grad_(True) for p in to_dev(scene, dev)]
    outs = render(rast, *leaves, distortion=True)
    assert len(outs) == 5
    rng = np.random.default_rng(51)
    g = torch.from_numpy(rng.normal(size=rast.total_pixels).astype(np.float32)).to(dev)
    (outs[4] * g).sum().backward()
    torch.cuda.synchronize()
    gouts = [np.concatenate([np.zeros((views[0].pixels, 9)),
                             g.cpu().numpy().astype(np.float64)[:, None]], axis=1)]
    st = oracle_settings(s)
    ref = oracle.backward(st, views, scene, gouts)
    scale = oracle.gradient_error_scale(st, views, scene, gouts)
    got = dict(means=leaves[0].grad.cpu().numpy(), scales=leaves[1].grad.cpu().numpy(),
               quats=leaves[2].grad.cpu().numpy(), opacities=leaves[3].grad.cpu().numpy(),
               sh=leaves[4].grad.cpu().numpy())
    grad_check(got, ref, scale, "autograd distortion")
