"""Pins of the oracle's normal-consistency regulariser (Eq. 24)."""
import numpy as np
import pytest

import oracle
from oracle_helpers import view


def _maps(seed, H=12, W=15):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    D = 3.0 + 0.05 * xx + 0.08 * yy + 0.02 * np.sin(xx + 2 * yy) + 0.01 * rng.normal(size=(H, W))
    N = rng.normal(size=(3, H, W)) * 0.3
    N[2] -= 0.6
    A = rng.uniform(0.2, 1.0, size=(H, W))
    return D, N, A


def test_plane_gives_plane_normal():
    # A planar surface n . X = d seen by a pinhole camera: the back-projected
    # depth map lies on the plane, so n~ is the plane normal facing the camera
    # (exactly, since central differences of points on a plane lie in it).
    v = view(20, 16, 18.0)
    m = np.array([0.3, -0.2, -1.0])
    m /= np.linalg.norm(m)
    d0 = -3.0
    H, W = 16, 20
    xs = (np.arange(W) + 0.5 - v.cx) / v.fx
    ys = (np.arange(H) + 0.5 - v.cy) / v.fy
    rdot = m[0] * xs[None, :] + m[1] * ys[:, None] + m[2]
    D = d0 / rdot                    # depth where the pixel ray meets the plane
    N = np.zeros((3, H, W))
    A = np.ones((H, W))
    N[:] = m[:, None, None]          # splat normals equal to the plane normal
    loss, gD, gN, gA = oracle.normal_consistency(v, D, N, A, 1.0)
    assert abs(loss) < 1e-12         # alpha - N . n~ = 1 - 1
    _, _, gN2, _ = oracle.normal_consistency(v, D, np.zeros_like(N), A, 1.0)
    nt = -gN2[:, 1:-1, 1:-1] * (H - 2) * (W - 2)
    np.testing.assert_allclose(nt, m[:, None, None] * np.ones((3, H - 2, W - 2)), atol=1e-12)


def test_gradient_matches_central_differences():
    v = view(15, 12, 14.0)
    D, N, A = _maps(3)
    loss, gD, gN, gA = oracle.normal_consistency(v, D, N, A, 5.0)
    rng = np.random.default_rng(0)
    for arr, g in ((D, gD), (N, gN), (A, gA)):
        for idx in rng.choice(arr.size, 25, replace=False):
            h = 1e-6 * max(1.0, abs(arr.flat[idx]))
            orig = arr.flat[idx]
            arr.flat[idx] = orig + h
            lp = oracle.normal_consistency(v, D, N, A, 5.0)[0]
            arr.flat[idx] = orig - h
            lm = oracle.normal_consistency(v, D, N, A, 5.0)[0]
            arr.flat[idx] = orig
            fd = (lp - lm) / (2 * h)
            assert g.flat[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_border_pixels_carry_no_loss():
    v = view(15, 12, 14.0)
    D, N, A = _maps(4)
    loss, gD, gN, gA = oracle.normal_consistency(v, D, N, A, 1.0)
    assert (gA[0] == 0).all() and (gA[-1] == 0).all() and (gA[:, 0] == 0).all()
    assert (gN[:, 0] == 0).all() and (gN[:, :, -1] == 0).all()
    # the border depths still receive gradient (they enter the differences)
    assert np.abs(gD[0, 1:-1]).max() > 0
