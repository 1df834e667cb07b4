"""GPU parity of TSDF fusion of median-depth maps (the mesh extraction of
Sec. 4.1) with the FP64 oracle.  Both sides fuse the same FP32 depth maps
(the rasterizer's median planes, or hand-made maps): the contributing-view
counts are integers and must match exactly, the fused values (means of
terms in [-1, 1], summed in FP32 on the GPU) within 1e-6; voxels whose
pixel lookup or truncation decision sits within rounding of a boundary
are excluded."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import device, say, to_dev

pytestmark = pytest.mark.gpu


def _settings(**kw):
    from paper_2406_01467_amd import Settings
    return Settings(**kw)


def _fuse_and_check(rast, depth, med_planes, views, origin, voxel, dims, trunc, label,
                    min_seen=0.05):
    import torch
    from paper_2406_01467_amd.tsdf import tsdf_fuse
    trunc = float(np.float32(trunc))  # the kernel holds it in FP32
    tsdf, weight = tsdf_fuse(rast, depth, origin, voxel, dims, trunc)
    torch.cuda.synchronize()
    got_t = tsdf.cpu().numpy().reshape(-1).astype(np.float64)
    got_w = weight.cpu().numpy().reshape(-1)
    ref_t, ref_w, frag = oracle.tsdf_fuse(views, med_planes, origin, voxel, dims, trunc,
                                          near=rast.settings.near_plane, return_fragile=True)
    keep = ~frag
    seen = (ref_w > 0).mean()
    say(f"  {label}: {ref_w.size} voxels, {seen:.3f} seen, max weight {ref_w.max():.0f}, "
        f"{frag.sum()} fragile")
    assert seen >= min_seen
    assert np.all(got_w == np.round(got_w))
    np.testing.assert_array_equal(got_w[keep], ref_w[keep])
    err = np.abs(got_t[keep] - ref_t[keep])
    assert err.max() <= 1e-6, (label, err.max())
    assert np.all(got_t[got_w == 0] == 0.0)


def _grid_around(means, n_vox):
    lo, hi = np.percentile(means, 2, axis=0), np.percentile(means, 98, axis=0)
    voxel = float((hi - lo).max() / n_vox)
    dims = tuple(int(np.ceil(e / voxel)) + 1 for e in (hi - lo))
    return lo.astype(np.float64), voxel, dims


def test_tsdf_of_rendered_median_depth_five_views():
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene = synth.make_scene_clusters(20000, seed=71, width=200, height=150, dist_range=(2, 8))
    views = synth.make_views_orbit(scene.means.mean(0), 9.0, 5, seed=72,
                                   size_range=((90, 240), (70, 180)))
    s = _settings(sh_degree=3)
    rast = Rasterizer(views, s, dev)
    maps = rast.forward(*to_dev(scene, dev))
    med = [maps.view_planes(rast, vi)["depth"][1].cpu().numpy() for vi in range(len(views))]
    assert all((m > 0).mean() > 0.05 for m in med)
    origin, voxel, dims = _grid_around(scene.means, 61)   # ragged: dims are not tile multiples
    _fuse_and_check(rast, maps.depth, med, views, origin, voxel, dims, 4 * voxel, "5 views")


def test_tsdf_hand_made_maps_with_holes_and_ragged_grid():
    import torch
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    centre = np.array([0.0, 0.0, 0.0])
    views = synth.make_views_orbit(centre, 3.0, 3, seed=73, sizes=[(64, 48), (57, 33), (80, 61)])
    rast = Rasterizer(views, _settings(sh_degree=0), dev)
    rng = np.random.default_rng(74)
    med, planes = [], []
    for v in views:
        D = rng.uniform(2.5, 3.5, (v.height, v.width)).astype(np.float32)
        D[rng.random(D.shape) < 0.2] = 0.0          # pixels with no surface
        med.append(D)
        planes.append(np.concatenate([np.zeros(v.pixels, np.float32), D.reshape(-1)]))
    depth = torch.from_numpy(np.concatenate(planes)).to(dev)
    dims = (37, 29, 23)
    voxel = 0.061
    origin = -0.5 * voxel * np.array(dims, np.float64)
    _fuse_and_check(rast, depth, med, views, origin, voxel, dims, 0.2, "hand-made maps")
    # one voxel grid, 1 x 1 x 1, and a grid outside every view
    _fuse_and_check(rast, depth, med, views, np.array([-0.013, -0.012, -0.011]), 0.02, (1, 1, 1),
                    0.2, "single voxel")
    _fuse_and_check(rast, depth, med, views, np.array([50.0, 50.0, 50.0]), 0.1, (5, 4, 3),
                    0.2, "unseen grid", min_seen=0.0)


def test_tsdf_rejects_bad_arguments():
    import torch
    from paper_2406_01467_amd import _lib
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    views = [synth.identity_view(32, 32)]
    rast = Rasterizer(views, _settings(sh_degree=0), dev)
    depth = torch.zeros(2 * 32 * 32, device=dev)
    out = torch.empty(8, device=dev)
    w = torch.empty(8, device=dev)
    for voxel, dims, trunc in [(0.0, (2, 2, 2), 0.1), (0.1, (0, 2, 2), 0.1),
                               (0.1, (2, 2, 2), 0.0), (float("nan"), (2, 2, 2), 0.1),
                               (0.1, (2048, 2048, 1025), 0.1)]:   # beyond 2^32 - 1 voxels
        with pytest.raises(RuntimeError):
            _lib.rade_tsdf_fuse(rast.settings, rast.views_c, rast.views_dev, depth, (0, 0, 0),
                                voxel, dims, trunc, out, w)


def test_tsdf_1600x1064_1m_median_depth():
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    scene, views = synth.make_workload("plain_1600x1064_1m")
    s = _settings(sh_degree=3)
    rast = Rasterizer(views, s, dev)
    maps = rast.forward(*to_dev(scene, dev))
    med = [maps.view_planes(rast, 0)["depth"][1].cpu().numpy()]
    origin, voxel, dims = _grid_around(scene.means, 127)
    _fuse_and_check(rast, maps.depth, med, views, origin, voxel, dims, 3 * voxel,
                    "1600x1064 1M", min_seen=0.01)
