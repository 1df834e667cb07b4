"""Pins of the oracle's exact per-pixel depth (Sec. 3.2.1, Eq. 5-7): the depth
of the maximum of the Gaussian along the ray through the pixel, as an
alternative to the affine depth plane of Eq. 4."""
import numpy as np
from scipy.optimize import minimize_scalar

import oracle
from oracle_helpers import rotation_wxyz, scene_from, view


def _maps(scene, v, exact=True, **kw):
    st = oracle.settings(depth_exact=exact, **kw)
    rec, _, flags, outs = oracle.forward(st, [v], scene)
    return rec[0], outs[0]


def _ray(v, px, py):
    return np.array([(px + 0.5 - np.float32(v.cx)) / np.float32(v.fx),
                     (py + 0.5 - np.float32(v.cy)) / np.float32(v.fy), 1.0])


def test_isotropic_gaussian_gives_the_foot_of_the_perpendicular():
    mean = np.array([0.3, -0.2, 3.0], np.float32)
    sc = scene_from([mean], [[0.12, 0.12, 0.12]], opac=[0.9])
    v = view(64, 64, 64.0)
    _, o = _maps(sc, v)
    a = o["alpha"]
    seen = np.nonzero(a > 0)[0]
    assert len(seen) > 100
    for idx in seen[::7]:
        px, py = idx % 64, idx // 64
        r = _ray(v, px, py)
        want = r @ mean.astype(np.float64) / (r @ r)   # camera z of the closest ray point
        np.testing.assert_allclose(o["depth_med"][idx], want, rtol=1e-12)
        np.testing.assert_allclose(o["depth_exp"][idx] / a[idx], want, rtol=1e-12)


def test_flat_gaussian_gives_the_ray_plane_intersection():
    q = np.array([0.8, 0.35, -0.3, 0.2])
    q /= np.linalg.norm(q)
    mean = np.array([-0.2, 0.1, 2.5], np.float32)
    sc = scene_from([mean], [[0.3, 0.2, 1e-5]], quats=[q], opac=[0.9])
    v = view(64, 64, 64.0)
    _, o = _maps(sc, v)
    n = rotation_wxyz(np.asarray(sc.quats[0], np.float64))[:, 2]   # the thin axis
    seen = np.nonzero(o["alpha"] > 0)[0]
    assert len(seen) > 200
    for idx in seen[::11]:
        r = _ray(v, idx % 64, idx // 64)
        want = (n @ mean.astype(np.float64)) / (n @ r)
        np.testing.assert_allclose(o["depth_med"][idx], want, rtol=1e-7)


def test_depth_is_the_maximum_along_the_ray_by_search():
    rng = np.random.default_rng(5)
    for trial in range(3):
        q = rng.normal(size=4)
        mean = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), rng.uniform(2, 4)],
                        np.float32)
        scales = np.exp(rng.normal(-2.5, 0.5, 3)).astype(np.float32)
        sc = scene_from([mean], [scales], quats=[q], opac=[0.95])
        v = view(48, 40, 50.0)
        _, o = _maps(sc, v)
        Rg = rotation_wxyz(np.asarray(sc.quats[0], np.float64))
        Sig = Rg @ np.diag(scales.astype(np.float64) ** 2) @ Rg.T
        Ai = np.linalg.inv(Sig)
        xc = mean.astype(np.float64)
        seen = np.nonzero(o["alpha"] > 0)[0]
        assert len(seen) > 20
        for idx in seen[:: max(1, len(seen) // 12)]:
            r = _ray(v, idx % 48, idx // 48)
            u = r / np.linalg.norm(r)
            f = lambda t: (t * u - xc) @ Ai @ (t * u - xc)  # noqa: E731
            t0 = u @ xc
            res = minimize_scalar(f, bounds=(t0 - 1.0, t0 + 1.0), method="bounded",
                                  options={"xatol": 1e-12})
            np.testing.assert_allclose(o["depth_med"][idx], res.x * u[2], rtol=1e-8)


def test_on_axis_first_order_is_the_affine_plane():
    """For a Gaussian on the optical axis, the derivative of the exact depth
    at its centre pixel equals p of Eq. 4 (the affine plane is the
    first-order form of the ray maximum there); a long focal length makes
    the central difference over one pixel accurate to ~1e-7."""
    q = np.array([0.9, 0.3, -0.2, 0.25])
    q /= np.linalg.norm(q)
    sc = scene_from([[0.0, 0.0, 3.0]], [[0.012, 0.006, 0.003]], quats=[q], opac=[0.9])
    v = view(64, 64, 4000.0, cx=32.5, cy=32.5)
    rec, o = _maps(sc, v)
    d = o["depth_med"].reshape(64, 64)
    assert d[32, 32] == np.float32(3.0)
    # dx = u_c - u: pixel 31 lies at dx = +1
    du = (d[32, 31] - d[32, 33]) / 2
    dv = (d[31, 32] - d[33, 32]) / 2
    np.testing.assert_allclose([du, dv], [rec[0, oracle.R["p0"]], rec[0, oracle.R["p1"]]],
                               rtol=1e-6)
    # off axis the two differ at first order (the plane is a local affine
    # approximation of the perspective rays); the Jacobian's field-of-view
    # clamp is lifted so that it plays no part
    sc_off = scene_from([[0.6, 0.0, 3.0]], [[0.012, 0.006, 0.003]], quats=[q], opac=[0.9])
    v_off = view(64, 64, 4000.0, cx=32.5 - 800.0, cy=32.5)
    rec_o, o_off = _maps(sc_off, v_off, fov_clamp=1e6)
    d_off = o_off["depth_med"].reshape(64, 64)
    du_off = (d_off[32, 31] - d_off[32, 33]) / 2
    assert abs(du_off - rec_o[0, oracle.R["p0"]]) > 1e-3 * abs(du_off)


def test_only_depth_maps_change():
    rng = np.random.default_rng(6)
    n = 40
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n),
                      rng.uniform(2.0, 4.0, n)], 1)
    sc = scene_from(means, np.exp(rng.normal(-2.5, 0.4, (n, 3))), quats=rng.normal(size=(n, 4)),
                    opac=rng.uniform(0.3, 0.9, n), rgb=rng.uniform(0, 1, (n, 3)))
    v = view(40, 32, 40.0)
    _, a = _maps(sc, v, exact=False)
    _, b = _maps(sc, v, exact=True)
    for k in ("color", "normal", "alpha", "t_final", "count", "last_id", "median_id"):
        np.testing.assert_array_equal(a[k], b[k])
    assert np.abs(a["depth_exp"] - b["depth_exp"]).max() > 0
    # the two depths agree at the centre and to first order: close overall
    np.testing.assert_allclose(b["depth_exp"], a["depth_exp"], rtol=0.05, atol=1e-3)
