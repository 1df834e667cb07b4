"""Pins of the oracle's 3D smoothing filter (the Mip-Splatting filter the
paper trains with, Sec. 4.1)."""
import numpy as np

import oracle
import synth
from oracle_helpers import view


def test_on_axis_rate_is_focal_over_depth():
    v = view(64, 48, 50.0)
    means = np.array([[0.0, 0.0, 3.0], [0.0, 0.0, 7.5]], np.float32)
    var = oracle.filter3d_var([v], means, scale=0.2)
    np.testing.assert_allclose(var, 0.2 * (means[:, 2].astype(np.float64) / 50.0) ** 2, rtol=1e-14)


def test_highest_rate_over_the_views_that_see_the_mean():
    near_view = view(64, 64, 64.0)                                   # z = 2 -> rate 32
    far_view = view(64, 64, 64.0, t=[0.0, 0.0, 4.0])                # z = 6 -> rate 10.7
    wide_view = view(64, 64, 16.0)                                   # rate 8
    behind = view(64, 64, 64.0, t=[0.0, 0.0, -5.0])                 # z = -3: not seen
    m = np.array([[0.0, 0.0, 2.0]], np.float32)
    var = oracle.filter3d_var([far_view, wide_view, near_view, behind], m, scale=0.3)
    np.testing.assert_allclose(var, 0.3 / 32.0 ** 2, rtol=1e-14)
    var = oracle.filter3d_var([far_view, wide_view], m, scale=0.3)
    np.testing.assert_allclose(var, 0.3 / (64.0 / 6.0) ** 2, rtol=1e-14)
    assert oracle.filter3d_var([behind], m)[0] == 0.0


def test_widened_image_decides_visibility():
    v = view(100, 80, 100.0)   # cx = 50: u = 100 x / z + 50
    z = 4.0
    # u = -10 (inside a 15 % margin of 100 px) and u = -20 (outside)
    xs = [(-10.0 - 50.0) * z / 100.0, (-20.0 - 50.0) * z / 100.0]
    m = np.array([[x, 0.0, z] for x in xs], np.float32)
    var = oracle.filter3d_var([v], m, scale=0.2, margin=0.15)
    assert var[0] > 0 and var[1] == 0.0


def test_filter_adds_isotropic_variance_and_keeps_the_integral():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(4)
    n = 50
    s = np.exp(rng.normal(-2.5, 0.7, (n, 3)))
    o = rng.uniform(0.1, 0.9, n)
    var = rng.uniform(0.0, 0.01, n)
    var[:5] = 0.0
    sf, of = oracle.filter3d_apply(s, o, var)
    for g in range(n):
        Rm = Rotation.random(random_state=g).as_matrix()
        S = Rm @ np.diag(s[g] ** 2) @ Rm.T
        Sf = Rm @ np.diag(sf[g] ** 2) @ Rm.T
        np.testing.assert_allclose(Sf, S + var[g] * np.eye(3), atol=1e-15)
    # integral of o exp(-x^T S^-1 x / 2) is o sqrt(det S) (2 pi)^(3/2)
    np.testing.assert_allclose(of * np.prod(sf, axis=1), o * np.prod(s, axis=1), rtol=1e-13)
    np.testing.assert_array_equal(sf[:5], s[:5])
    np.testing.assert_array_equal(of[:5], o[:5])


def test_adjoint_matches_central_differences():
    rng = np.random.default_rng(6)
    n = 20
    s = np.exp(rng.normal(-2.5, 0.7, (n, 3))) * rng.choice([-1, 1], (n, 3))
    o = rng.uniform(0.1, 0.9, n)
    var = rng.uniform(1e-4, 0.01, n)
    gs, go = rng.normal(size=(n, 3)), rng.normal(size=n)

    def L(ss, oo):
        a, b = oracle.filter3d_apply(ss, oo, var)
        return float((a * gs).sum() + (b * go).sum())

    ds, do = oracle.filter3d_apply_bwd(s, o, var, gs, go)
    for g in range(n):
        for k in range(3):
            h = 1e-6 * abs(s[g, k])
            sp, sm = s.copy(), s.copy()
            sp[g, k] += h
            sm[g, k] -= h
            fd = (L(sp, o) - L(sm, o)) / (2 * h)
            assert abs(fd - ds[g, k]) <= 1e-6 * (abs(ds[g, k]) + 1e-3), (g, k, fd, ds[g, k])
        op, om = o.copy(), o.copy()
        op[g] += 1e-6
        om[g] -= 1e-6
        fd = (L(s, op) - L(s, om)) / 2e-6
        assert abs(fd - do[g]) <= 1e-7 * (abs(do[g]) + 1.0)


def test_cluster_scene_orbit_views_have_finite_positive_variance():
    scene = synth.make_scene_clusters(2000, seed=3, width=200, height=150, dist_range=(2, 8))
    views = synth.make_views_orbit(scene.means.mean(0), 10.0, 4, seed=4,
                                   sizes=[(200, 150)] * 4)
    var, frag = oracle.filter3d_var(views, scene.means, return_fragile=True)
    assert np.isfinite(var).all() and (var >= 0).all()
    assert (var > 0).mean() > 0.5 and frag.sum() == 0
