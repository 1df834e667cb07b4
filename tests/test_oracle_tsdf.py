"""Pins of the oracle's TSDF fusion of median-depth maps (Sec. 4.1, Mesh
Extraction)."""
import numpy as np

import oracle
from oracle_helpers import view


def _grid():
    # 8 x 8 x 16 voxels of 0.05 in front of the camera, z in [2.0, 2.8]
    return np.array([-0.2, -0.2, 2.0]), 0.05, (8, 8, 16)


def test_fronto_parallel_plane_closed_form():
    v = view(64, 64, 64.0)
    origin, h, dims = _grid()
    D = np.full((64, 64), 2.37)
    trunc = 0.15
    tsdf, w = oracle.tsdf_fuse([v], [D], origin, h, dims, trunc)
    z = origin[2] + (np.arange(dims[2]) + 0.5) * h
    s = 2.37 - z
    want_w = (s >= -trunc).astype(float)
    want = np.where(s >= -trunc, np.minimum(1.0, s / trunc), 0.0)
    nxy = dims[0] * dims[1]
    for k in range(dims[2]):
        np.testing.assert_allclose(tsdf[k * nxy:(k + 1) * nxy], want[k], rtol=1e-12, atol=1e-15)
        np.testing.assert_array_equal(w[k * nxy:(k + 1) * nxy], want_w[k])
    # the zero crossing sits at the surface depth
    k0 = np.argmin(np.abs(s))
    assert abs(s[k0]) <= h / 2


def test_views_average_and_unseen_voxels():
    v1 = view(64, 64, 64.0)
    v2 = view(64, 64, 64.0, t=[0.0, 0.0, 0.125])   # same axis, 0.125 further away
    origin, h, dims = _grid()
    D1, D2 = np.full((64, 64), 2.4), np.full((64, 64), 2.525)   # the same plane z = 2.4
    tsdf, w = oracle.tsdf_fuse([v1, v2], [D1, D2], origin, h, dims, 0.2)
    one, w1 = oracle.tsdf_fuse([v1], [D1], origin, h, dims, 0.2)
    np.testing.assert_allclose(tsdf[w == 2], one[w == 2], rtol=1e-12, atol=1e-15)
    assert w.max() == 2
    # no surface (depth 0) -> no contribution
    tsdf0, w0 = oracle.tsdf_fuse([v1], [np.zeros((64, 64))], origin, h, dims, 0.2)
    assert w0.max() == 0 and np.all(tsdf0 == 0)
    # a grid behind the camera is never seen
    tsdf_b, w_b = oracle.tsdf_fuse([v1], [D1], np.array([-0.2, -0.2, -3.0]), h, dims, 0.2)
    assert w_b.max() == 0


def test_pixel_lookup_follows_the_projection():
    # depth map with one value per image column: the voxel column seen
    # through pixel column c reads depth 2 + 0.01 c
    v = view(64, 64, 64.0)
    origin, h, dims = _grid()
    D = np.tile(2.0 + 0.01 * np.arange(64), (64, 1))
    tsdf, w = oracle.tsdf_fuse([v], [D], origin, h, dims, 10.0)
    nx, ny, nz = dims
    for idx in [0, 77, 400, nx * ny * nz - 1]:
        i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
        X = origin + (np.array([i, j, k]) + 0.5) * h
        u = 64.0 * X[0] / X[2] + 32.0
        d = 2.0 + 0.01 * np.floor(u)
        np.testing.assert_allclose(tsdf[idx], min(1.0, (d - X[2]) / 10.0), rtol=1e-12)
