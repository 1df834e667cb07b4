"""GPU parity of the 3D smoothing filter (the Mip-Splatting filter of
Sec. 4.1) with the FP64 oracle: the per-Gaussian variance from the cameras,
the transform of scales and opacities, its adjoint, and the whole path
(filter -> rasterizer -> gradients through the filter)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import device, grad_check, oracle_settings, say, to_dev

pytestmark = pytest.mark.gpu


def _settings(**kw):
    from paper_2406_01467_amd import Settings
    return Settings(**kw)


def _scene_views(n=20000, seed=61):
    scene = synth.make_scene_clusters(n, seed=seed, width=200, height=150, dist_range=(2, 8))
    views = synth.make_views_orbit(scene.means.mean(0), 9.0, 5, seed=seed + 1,
                                   size_range=((60, 240), (40, 180)))
    return scene, views


def test_filter_variance_matches_oracle():
    import torch
    from paper_2406_01467_amd.filter3d import filter3d_var
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = _scene_views()
    s = _settings(sh_degree=3)
    rast = Rasterizer(views, s, dev)
    means = torch.from_numpy(scene.means).to(dev)
    got = filter3d_var(rast, means, scale=0.2, margin=0.15).cpu().numpy().astype(np.float64)
    ref, frag = oracle.filter3d_var(views, scene.means, near=s.near_plane, scale=0.2,
                                    margin=0.15, return_fragile=True)
    keep = ~frag
    say("filter var:", (ref > 0).sum(), "seen of", scene.n, "; fragile", frag.sum())
    assert (ref > 0).sum() > 0.5 * scene.n
    np.testing.assert_array_equal(got[keep] > 0, ref[keep] > 0)
    np.testing.assert_allclose(got[keep], ref[keep], rtol=1e-6, atol=0)


def test_filter_transform_and_adjoint_match_oracle():
    import torch
    from paper_2406_01467_amd import _lib
    dev = device()
    rng = np.random.default_rng(62)
    n = 100003  # not a multiple of the block size
    s = (np.exp(rng.normal(-3.0, 0.8, (n, 3))) * rng.choice([-1, 1], (n, 3))).astype(np.float32)
    o = rng.uniform(0.02, 0.98, n).astype(np.float32)
    var = rng.uniform(0.0, 0.01, n).astype(np.float32)
    var[::7] = 0.0
    gs = rng.normal(size=(n, 3)).astype(np.float32)
    go = rng.normal(size=n).astype(np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    S, O, F, GS, GO = t(s), t(o), t(var), t(gs), t(go)
    s_out, o_out = torch.empty_like(S), torch.empty_like(O)
    _lib.rade_filter3d_apply(n, S, O, F, s_out, o_out)
    ds, do = torch.empty_like(S), torch.empty_like(O)
    _lib.rade_filter3d_apply_bwd(n, S, O, F, GS, GO, ds, do)
    # in place: gradients written over the upstream buffers
    GS2, GO2 = GS.clone(), GO.clone()
    _lib.rade_filter3d_apply_bwd(n, S, O, F, GS2, GO2, GS2, GO2)
    torch.cuda.synchronize()
    rs, ro = oracle.filter3d_apply(s, o, var)
    rds, rdo = oracle.filter3d_apply_bwd(s, o, var, gs, go)
    np.testing.assert_allclose(s_out.cpu().numpy(), rs, rtol=2e-7)
    np.testing.assert_allclose(o_out.cpu().numpy(), ro, rtol=1e-6)
    # each gradient is a sum of two products: bound by the sum of their sizes
    sf = np.sqrt(s.astype(np.float64) ** 2 + var[:, None])
    mag = np.abs(gs * s / sf) + np.abs(go * ro)[:, None] * var[:, None] / np.abs(s * sf * sf)
    assert np.all(np.abs(ds.cpu().numpy() - rds) <= 1e-5 * mag + 1e-30)
    np.testing.assert_allclose(do.cpu().numpy(), rdo, rtol=1e-6, atol=1e-30)
    assert torch.equal(GS2, ds) and torch.equal(GO2, do)


def test_filtered_render_gradients_through_the_filter():
    import torch
    from paper_2406_01467_amd.filter3d import apply_filter3d, filter3d_var
    from paper_2406_01467_amd.raster import Rasterizer, render
    dev = device()
    scene = synth.make_scene_clusters(3000, seed=63, width=80, height=64, dist_range=(2, 5))
    views = [synth.identity_view(80, 64)] + synth.make_views_orbit(
        scene.means.mean(0), 4.0, 1, seed=64, sizes=[(64, 56)])
    s = _settings(sh_degree=3)
    rast = Rasterizer(views, s, dev)
    leaves = [p.detach().clone().requires_grad_(True) for p in to_dev(scene, dev)]
    var = filter3d_var(rast, leaves[0].detach())
    fs, fo = apply_filter3d(leaves[1], leaves[3], var)
    outs = render(rast, leaves[0], fs, leaves[2], fo, leaves[4])
    rng = np.random.default_rng(65)
    P = rast.total_pixels
    ups = [rng.normal(size=k * P).astype(np.float32) for k in (3, 2, 3, 1)]
    loss = sum((o * torch.from_numpy(u).to(dev)).sum() for o, u in zip(outs, ups))
    loss.backward()
    torch.cuda.synchronize()
    # oracle: filter in FP64 from the same variance (rounded as the kernel
    # stores it), render the filtered scene, chain its scale and opacity
    # gradients back through the filter
    var_h = var.cpu().numpy()
    rs, ro = oracle.filter3d_apply(scene.scales, scene.opacities, var_h)
    fscene = synth.Scene(scene.means, rs.astype(np.float32), scene.quats,
                         ro.astype(np.float32), scene.sh, scene.sh_degree)
    gouts = []
    for vi, v in enumerate(views):
        o, Pv = rast.views_c[vi].pix_offset, v.pixels
        g = np.zeros((Pv, 9))
        g[:, 0:3] = ups[0][3 * o: 3 * o + 3 * Pv].reshape(3, Pv).T
        g[:, 3:5] = ups[1][2 * o: 2 * o + 2 * Pv].reshape(2, Pv).T
        g[:, 5:8] = ups[2][3 * o: 3 * o + 3 * Pv].reshape(3, Pv).T
        g[:, 8] = ups[3][o: o + Pv]
        gouts.append(g)
    st = oracle_settings(s)
    ref = oracle.backward(st, views, fscene, gouts)
    scale = oracle.gradient_error_scale(st, views, fscene, gouts)
    ds, do = oracle.filter3d_apply_bwd(scene.scales, scene.opacities, var_h, ref["scales"],
                                       ref["opacities"])
    ds_abs, do_abs = oracle.filter3d_apply_bwd(np.abs(scene.scales), scene.opacities, var_h,
                                               scale["scales"], scale["opacities"])
    ref["scales"], ref["opacities"] = ds, do
    scale["scales"], scale["opacities"] = np.abs(ds_abs), np.abs(do_abs)
    got = dict(means=leaves[0].grad.cpu().numpy(), scales=leaves[1].grad.cpu().numpy(),
               quats=leaves[2].grad.cpu().numpy(), opacities=leaves[3].grad.cpu().numpy(),
               sh=leaves[4].grad.cpu().numpy())
    grad_check(got, ref, scale, "render through the 3D filter")
