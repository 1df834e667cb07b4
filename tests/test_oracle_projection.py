"""Pins of the oracle's projection against facts fixed by geometry, the paper's
own identities and library routines (no retyping of the oracle's formulas)."""
import numpy as np
import pytest

import oracle
from oracle import R
from oracle_helpers import pixel_index, rotation_wxyz, scene_from, view


def _proj(s, v, scene):
    rec, rect, flags = oracle.project(s, [v], scene)
    return rec[0], rect[0], flags[0]


def _ray_dir(v, u, w):
    return np.array([(u - v.cx) / v.fx, (w - v.cy) / v.fy, 1.0])


def test_centre_is_pinhole_projection():
    # The splat centre is the pinhole image of the mean (Sec. 3.2, u_c, v_c).
    v = view(96, 80, 70.0)
    means = [[0.3, -0.2, 2.5], [-0.7, 0.4, 3.1], [0.0, 0.0, 1.0]]
    sc = scene_from(means, [[0.05] * 3] * 3)
    rec, _, _ = _proj(oracle.settings(), v, sc)
    for i, m in enumerate(means):
        m = np.asarray(m, np.float32).astype(np.float64)
        assert rec[i, R["uc"]] == pytest.approx(70.0 * m[0] / m[2] + 48.0, abs=1e-12)
        assert rec[i, R["vc"]] == pytest.approx(70.0 * m[1] / m[2] + 40.0, abs=1e-12)
        assert rec[i, R["z"]] == pytest.approx(m[2], abs=1e-15)


def test_isotropic_plane_and_normal():
    # Isotropic Gaussian: Sigma' has no (uv, t) coupling, so q = p = 0 and the
    # normal is the unit vector from the centre to the camera (Eq. 13, 21-22).
    v = view(64, 64, 64.0)
    means = [[0.4, -0.3, 3.0], [-0.8, 0.6, 2.2], [0.1, 0.9, 4.0]]
    for dil in (0.0, 0.3):
        sc = scene_from(means, [[0.07] * 3] * 3)
        rec, _, flags = _proj(oracle.settings(dilation=dil), v, sc)
        for i, m in enumerate(means):
            m = np.asarray(m, np.float32).astype(np.float64)
            assert abs(rec[i, R["q0"]]) < 1e-12 and abs(rec[i, R["q1"]]) < 1e-12
            n = rec[i, [R["n0"], R["n1"], R["n2"]]]
            np.testing.assert_allclose(n, -m / np.linalg.norm(m), atol=1e-12)


def _perspective_tstar(v, Sigma_c, xc, u, w):
    """Eq. 7: maximiser of the Gaussian along the camera ray of pixel (u, w),
    measured as distance from the camera centre."""
    d = _ray_dir(v, u, w)
    d /= np.linalg.norm(d)
    A = np.linalg.inv(Sigma_c)
    return float(d @ A @ xc / (d @ A @ d))


@pytest.mark.parametrize("seed", range(6))
def test_plane_slope_matches_perspective_maximiser(seed):
    # The ray-space plane t* = t_c + q (u_c - u, v_c - v) (Eq. 12-13) is the
    # local affine approximation of the exact maximiser along each camera ray
    # (Eq. 7); both agree to first order at the splat centre.  Central
    # differences of Eq. 7 (computed from Sigma through scipy's rotation, not
    # through the oracle's formulas) pin q, the Jacobian's third row and
    # Sigma' for general anisotropic Gaussians.
    rng = np.random.default_rng(100 + seed)
    v = view(200, 160, 180.0)
    xc = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4), rng.uniform(2.0, 4.0)])
    scales = np.exp(rng.normal(-2.5, 0.6, 3))
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    sc = scene_from([xc], [scales], [q], opac=[0.9])
    xc64 = sc.means[0].astype(np.float64)
    Rg = rotation_wxyz(sc.quats[0])
    Sig = Rg @ np.diag(sc.scales[0].astype(np.float64) ** 2) @ Rg.T
    rec, _, flags = _proj(oracle.settings(dilation=0.0), v, sc)
    assert not flags[0] & oracle.F_DEGENERATE
    uc, vc = rec[0, R["uc"]], rec[0, R["vc"]]
    h = 1e-3
    for k, (du, dw) in enumerate([(h, 0.0), (0.0, h)]):
        # Delta = u_c - u, so pixel u = u_c - Delta.
        tp = _perspective_tstar(v, Sig, xc64, uc - du, vc - dw)
        tm = _perspective_tstar(v, Sig, xc64, uc + du, vc + dw)
        slope = (tp - tm) / (2 * h)
        assert rec[0, R["q0" if k == 0 else "q1"]] == pytest.approx(slope, rel=1e-6, abs=1e-9)
    # At the centre ray, Eq. 7 gives the distance of the centre (t_c).
    assert _perspective_tstar(v, Sig, xc64, uc, vc) == pytest.approx(np.linalg.norm(xc64), rel=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_thin_disk_normal_and_on_axis_depth_plane(seed):
    # A very flat Gaussian is a disk: its intersection plane is the disk plane,
    # so the normal is the disk normal m facing the camera (Eq. 21-22).  On the
    # optical axis the depth slope p of a plane with normal m through (0,0,Z)
    # is Z (m_x, m_y) / (f m_z) (first-order pinhole geometry).
    rng = np.random.default_rng(7 + seed)
    v = view(128, 128, 150.0)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    eps = 1e-5
    s = [0.2, 0.15, 0.2 * eps]
    for xc in ([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), 2.5], [0.0, 0.0, 3.0]):
        sc = scene_from([xc], [s], [q], opac=[0.9])
        Rg = rotation_wxyz(sc.quats[0])
        m = Rg[:, 2]  # the thin axis is the disk normal
        x64 = sc.means[0].astype(np.float64)
        rec, _, flags = _proj(oracle.settings(dilation=0.0), v, sc)
        n = rec[0, [R["n0"], R["n1"], R["n2"]]]
        expect = -np.sign(m @ x64) * m
        np.testing.assert_allclose(n, expect, atol=1e-6)
        assert n @ x64 < 0
        if xc[0] == 0.0 and xc[1] == 0.0:
            Z = x64[2]
            p_expect = Z * np.array([m[0], m[1]]) / (150.0 * m[2])
            np.testing.assert_allclose(rec[0, [R["p0"], R["p1"]]], p_expect, rtol=1e-6, atol=1e-12)


def test_footprint_is_jacobian_pushforward():
    # Eq. 2: the 2x2 footprint is J2 Sigma_c J2^T (+ dilation) with J2 the
    # Jacobian of the pinhole map; here J2 comes from central differences of
    # the pinhole map, Sigma from scipy's rotation.
    rng = np.random.default_rng(3)
    v = view(120, 90, 100.0)
    for _ in range(5):
        xc = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.3, 0.3), rng.uniform(1.5, 3.0)])
        scales = np.exp(rng.normal(-2.5, 0.5, 3))
        q = rng.normal(size=4)
        sc = scene_from([xc], [scales], [q / np.linalg.norm(q)], opac=[0.9])
        x = sc.means[0].astype(np.float64)
        Rg = rotation_wxyz(sc.quats[0])
        Sig = Rg @ np.diag(sc.scales[0].astype(np.float64) ** 2) @ Rg.T

        def pin(p):
            return np.array([100.0 * p[0] / p[2] + 60.0, 100.0 * p[1] / p[2] + 45.0])

        J2 = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-6
            J2[:, k] = (pin(x + e) - pin(x - e)) / 2e-6
        B = J2 @ Sig @ J2.T + 0.3 * np.eye(2)
        rec, _, _ = _proj(oracle.settings(dilation=0.3), v, sc)
        np.testing.assert_allclose([rec[0, R["B00"]], rec[0, R["B01"]], rec[0, R["B11"]]],
                                   [B[0, 0], B[0, 1], B[1, 1]], rtol=1e-7)
        conic = np.linalg.inv(B)
        np.testing.assert_allclose([rec[0, R["a"]], rec[0, R["b"]], rec[0, R["c"]]],
                                   [conic[0, 0], conic[0, 1], conic[1, 1]], rtol=1e-7)


def test_world_to_camera_transform():
    # The same Gaussian seen from a moved camera: the record equals that of
    # the Gaussian moved by the inverse motion under the identity camera
    # (Eq. 2, W).  Degree 0 colour, so the view direction does not matter.
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(11)
    Rw = Rotation.from_rotvec([0.2, -0.3, 0.1]).as_matrix().astype(np.float32)
    t = np.array([0.1, -0.2, 0.5], np.float32)
    means_cam = rng.uniform(-0.5, 0.5, (20, 3)) + np.array([0, 0, 3.0])
    Rw64, t64 = Rw.astype(np.float64), t.astype(np.float64)
    means_world = (means_cam - t64) @ Rw64  # R^T (x - t)
    q = rng.normal(size=(20, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    # Rotate the Gaussian frames by R^T as well, so camera-frame shapes match.
    Rq = Rotation.from_matrix(Rw64.T)
    qw = []
    for qi in q:
        r = Rq * Rotation.from_quat([qi[1], qi[2], qi[3], qi[0]])
        x, y, z, w = r.as_quat()
        qw.append([w, x, y, z])
    scales = np.exp(rng.normal(-3, 0.4, (20, 3)))
    s = oracle.settings()
    a = scene_from(means_world, scales, qw, opac=np.full(20, 0.7))
    b = scene_from(means_cam, scales, q, opac=np.full(20, 0.7))
    ra, _, _ = _proj(s, view(64, 64, 64.0, R=Rw, t=t), a)
    # b is built from float32 copies; compare with tolerance set by the FP32
    # rounding of the moved inputs (~1e-7 relative).
    rb, _, _ = _proj(s, view(64, 64, 64.0), b)
    for f in ("uc", "vc", "z", "a", "b", "c", "p0", "p1", "n0", "n1", "n2"):
        np.testing.assert_allclose(ra[:, R[f]], rb[:, R[f]], rtol=2e-5, atol=2e-5, err_msg=f)


@pytest.mark.parametrize("alpha_min", [1.0 / 255.0, 1e-3, 0.05])
def test_support_rect_is_conservative_and_tight(alpha_min):
    # The pixel rect contains every pixel the per-pixel rule can blend --
    # power <= cut (3 sigma) and alpha = o e^-power >= alpha_min, evaluated
    # here from the definition, not from the oracle's support tau -- and
    # extends at most one pixel beyond the ellipse's exact bounding box.
    # Opacities at or below alpha_min leave no such pixel: those Gaussians
    # are culled.
    rng = np.random.default_rng(5)
    v = view(80, 70, 80.0)
    n = 60
    means = rng.uniform(-0.6, 0.6, (n, 3)) + np.array([0, 0, 2.5])
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = rng.uniform(0.0005, 1, n)
    opac[:4] = [alpha_min * 0.999, alpha_min * 1.001, alpha_min * 1.5, alpha_min * 3.0]
    sc = scene_from(means, np.exp(rng.normal(-3.0, 0.6, (n, 3))), q, opac=opac)
    s = oracle.settings(alpha_min=alpha_min)
    rec, rect, flags = _proj(s, v, sc)
    o32 = sc.opacities.astype(np.float64)
    assert (((flags & oracle.F_CULLED) != 0) == (o32 <= alpha_min)).all()
    yy, xx = np.mgrid[0:v.height, 0:v.width]
    for g in range(n):
        if flags[g] & oracle.F_CULLED:
            continue
        r = rec[g]
        dx = r[R["uc"]] - (xx + 0.5)
        dy = r[R["vc"]] - (yy + 0.5)
        power = 0.5 * (r[R["a"]] * dx * dx + 2 * r[R["b"]] * dx * dy + r[R["c"]] * dy * dy)
        inside = (power <= 4.5) & (o32[g] * np.exp(-power) >= alpha_min)
        assert np.isclose(r[R["tau"]], min(4.5, np.log(o32[g] / alpha_min)), rtol=1e-14)
        if inside.any():
            assert flags[g] & oracle.F_VISIBLE
            ys, xs = np.nonzero(inside)
            x0, x1, y0, y1 = rect[g]
            assert x0 <= xs.min() and xs.max() <= x1 and y0 <= ys.min() and ys.max() <= y1
            # tight: exact bbox half-width sqrt(2 tau B00) + one pixel slack
            rx = np.sqrt(2 * r[R["tau"]] * r[R["B00"]])
            assert x0 >= np.floor(r[R["uc"]] - rx - 0.5) - 1 or x0 == 0
            assert x1 <= np.ceil(r[R["uc"]] + rx - 0.5) + 1 or x1 == v.width - 1


def test_cull_rules():
    v = view()
    sc = scene_from([[0, 0, 0.1], [0, 0, 3], [0, 0, 3], [np.nan, 0, 3], [0, 0, 3]],
                    [[0.1] * 3] * 5, opac=[0.5, 0.5, 1.0 / 255.0 * 0.9, 0.5, 0.5])
    sc.quats[4] = 0.0
    _, _, flags = _proj(oracle.settings(), v, sc)
    assert [bool(f & oracle.F_CULLED) for f in flags] == [True, False, True, True, True]


@pytest.mark.parametrize("seed", range(3))
def test_ray_space_maxima_are_coplanar(seed):
    """Under the local affine projection (Sec. 3.2.2), the maximum of the
    ray-space Gaussian along t at pixel offset D = (u_c - u, v_c - v) lies
    on the plane t = t_c + q . D (Eq. 12-17) for any D, not only to first
    order: a bounded 1D search of the Gaussian built here from J and Sigma
    (J from the pinhole derivatives and t = |x|, Sigma from scipy's
    rotation) against the oracle's q, at offsets up to 20 pixels."""
    from scipy.optimize import minimize_scalar
    rng = np.random.default_rng(300 + seed)
    f = 160.0
    v = view(200, 160, f)
    xc = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), rng.uniform(2.0, 4.0)])
    scales = np.exp(rng.normal(-2.5, 0.6, 3))
    q = rng.normal(size=4)
    sc = scene_from([xc], [scales], [q / np.linalg.norm(q)], opac=[0.9])
    rec, _, flags = _proj(oracle.settings(dilation=0.0, fov_clamp=1e6), v, sc)
    assert not flags[0] & oracle.F_DEGENERATE
    x, y, z = sc.means[0].astype(np.float64)
    t = np.sqrt(x * x + y * y + z * z)
    J = np.array([[f / z, 0.0, -f * x / z**2], [0.0, f / z, -f * y / z**2], [x / t, y / t, z / t]])
    Rg = rotation_wxyz(sc.quats[0])
    Sig = Rg @ np.diag(sc.scales[0].astype(np.float64) ** 2) @ Rg.T
    A = np.linalg.inv(J @ Sig @ J.T)
    qv = np.array([rec[0, R["q0"]], rec[0, R["q1"]]])
    for D in rng.uniform(-20, 20, (8, 2)):
        def energy(tt):
            w = np.array([-D[0], -D[1], tt - t])   # (u - u_c, v - v_c, t - t_c)
            return w @ A @ w
        res = minimize_scalar(energy, bounds=(t - 5.0, t + 5.0), method="bounded",
                              options={"xatol": 1e-13})
        assert res.x == pytest.approx(t + qv @ D, rel=1e-10, abs=1e-10)


def test_rigid_motion_invariance():
    """Rotating and translating the Gaussians and the camera by one rigid
    motion leaves every map unchanged (SH degree 0: colour does not depend
    on the view direction); FP32 storage of the moved inputs perturbs the
    maps at the 1e-6 level, pixels on a discrete threshold excepted."""
    import synth
    from scipy.spatial.transform import Rotation
    scene = synth.make_scene_uniform_cube(200, seed=11, sh_degree=0)
    rng = np.random.default_rng(12)
    Q = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    s = np.array([0.3, -0.2, 0.5])
    means = scene.means.astype(np.float64) @ Q.T + s
    rot = Rotation.from_matrix(Q) * Rotation.from_quat(
        np.concatenate([scene.quats[:, 1:], scene.quats[:, :1]], axis=1).astype(np.float64))
    qxyzw = rot.as_quat()
    quats = np.concatenate([qxyzw[:, 3:], qxyzw[:, :3]], axis=1)
    moved = scene_from(means, scene.scales, quats, scene.opacities, sh=scene.sh, degree=0)
    v0 = view(48, 48, 48.0)
    v1 = view(48, 48, 48.0, R=np.eye(3) @ Q.T, t=-(Q.T @ s))
    st = oracle.settings(sh_degree=0)
    _, _, _, oa = oracle.forward(st, [v0], scene)
    _, _, _, ob = oracle.forward(st, [v1], moved)
    keep = ((oa[0]["fragile"] | ob[0]["fragile"]) & 1) == 0
    assert keep.mean() > 0.98
    for k in ("color", "depth_exp", "normal", "alpha"):
        a = np.asarray(oa[0][k]).reshape(len(keep), -1)[keep]
        b = np.asarray(ob[0][k]).reshape(len(keep), -1)[keep]
        np.testing.assert_allclose(b, a, rtol=0, atol=2e-4 * max(1.0, np.abs(a).max()))
    # and the maps are not trivially empty
    assert oa[0]["alpha"].max() > 0.5
