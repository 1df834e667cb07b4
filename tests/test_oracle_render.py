"""Pins of the oracle's colour and compositing: real SH against scipy, closed
forms of Eq. 3 / Eq. 4, telescoping, invariances, the stop and median rules."""
import numpy as np
import pytest

import oracle
from oracle import R
from oracle_helpers import pixel_index, scene_from, view


def _real_sh_scipy(l, m, d):
    """Real SH from scipy's complex Y_l^m (Condon-Shortley phase included):
    sqrt(2) Re Y_l^m for m > 0, sqrt(2) Im Y_l^|m| for m < 0, Y_l^0."""
    from scipy.special import sph_harm_y
    x, y, z = d
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    if m == 0:
        return float(np.real(sph_harm_y(l, 0, theta, phi)))
    c = sph_harm_y(l, abs(m), theta, phi)
    return float(np.sqrt(2.0) * (np.real(c) if m > 0 else np.imag(c)))


def test_sh_basis_matches_scipy():
    # Colour channel 0 with a single SH coefficient 0.1 at index j reads
    # 0.1 * Y_j(dir) + 0.5; the direction is from the camera centre to the mean.
    rng = np.random.default_rng(0)
    v = view(64, 64, 64.0)
    dirs = rng.normal(size=(12, 3))
    dirs[:, 2] = np.abs(dirs[:, 2]) + 0.5
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    means = 3.0 * dirs
    j = 0
    for l in range(4):
        for m in range(-l, l + 1):
            sh = np.zeros((12, 16, 3), np.float32)
            sh[:, j, 0] = 0.1
            sc = scene_from(means, [[0.05] * 3] * 12, opac=np.full(12, 0.5), sh=sh, degree=3)
            rec, _, _ = oracle.project(oracle.settings(sh_degree=3), [v], sc)
            for i in range(12):
                d = sc.means[i].astype(np.float64)
                d /= np.linalg.norm(d)
                got = (rec[0, i, R["r"]] - 0.5) / 0.1
                assert got == pytest.approx(_real_sh_scipy(l, m, d), abs=1e-6), (l, m)
            j += 1


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre x uniform quadrature of Y_i Y_j over the sphere.
    v = view(64, 64, 64.0)
    nt, nphi = 16, 32
    xs, ws = np.polynomial.legendre.leggauss(nt)
    phis = np.arange(nphi) * 2 * np.pi / nphi
    dirs, wts = [], []
    for x, w in zip(xs, ws):
        for ph in phis:
            st = np.sqrt(1 - x * x)
            dirs.append([st * np.cos(ph), st * np.sin(ph), x])
            wts.append(w * 2 * np.pi / nphi)
    dirs = np.array(dirs)
    wts = np.array(wts)
    # Put the camera at the origin and the means on the unit sphere around it;
    # keep them in front (z > near) by moving the camera back along -z and
    # measuring directions from the camera centre: C = -R^T t = (0,0,-10).
    n = dirs.shape[0]
    Y = np.zeros((16, n))
    for j in range(16):
        sh = np.zeros((n, 16, 3), np.float32)
        sh[:, j, 0] = 0.1
        means = dirs + np.array([0, 0, -10.0])
        sc = scene_from(means, [[0.05] * 3] * n, opac=np.full(n, 0.5), sh=sh, degree=3)
        rec, _, flags = oracle.project(oracle.settings(sh_degree=3, near=-1e9),
                                       [view(64, 64, 64.0, t=[0, 0, 10.0])], sc)
        Y[j] = (rec[0, :, R["r"]] - 0.5) / 0.1
    G = (Y * wts[None, :]) @ Y.T
    np.testing.assert_allclose(G, np.eye(16), atol=2e-5)


def _single(o, mean, s, rgb, dil=0.3, px=32, py=32, bg=(0.0, 0.0, 0.0)):
    v = view(64, 64, 64.0)
    sc = scene_from([mean], [[s] * 3], opac=[o], rgb=[rgb])
    st = oracle.settings(dilation=dil, bg=bg)
    rec, rect, flags, outs = oracle.forward(st, [v], sc, pixels=[pixel_index(v, [px], [py])])
    return rec[0][0], outs[0]


def test_single_gaussian_closed_form():
    # Eq. 3 with one splat on the optical axis: alpha = o exp(-|d|^2 / (2 s2))
    # with s2 = (f sigma / z)^2 + dilation; C = alpha c + (1 - alpha) bg;
    # depth = alpha z (p = 0); normal = alpha (0, 0, -1).
    o, z, sig = 0.8, 3.0, 0.1
    for px, py in ((32, 32), (33, 31), (30, 34)):
        rec, out = _single(o, [0.0, 0.0, z], sig, [0.2, 0.4, 0.9], px=px, py=py, bg=(0.1, 0.2, 0.3))
        s2 = (64.0 * float(np.float32(sig)) / z) ** 2 + 0.3
        d2 = (32.0 - px - 0.5) ** 2 + (32.0 - py - 0.5) ** 2
        a = float(np.float32(o)) * np.exp(-0.5 * d2 / s2)
        sh0 = ((np.array([0.2, 0.4, 0.9]) - 0.5) * 2 * np.sqrt(np.pi)).astype(np.float32)
        rgb = sh0.astype(np.float64) * 0.5 / np.sqrt(np.pi) + 0.5
        np.testing.assert_allclose(out["alpha"][0], a, rtol=1e-12)
        np.testing.assert_allclose(out["color"][0], a * rgb + (1 - a) * np.array([0.1, 0.2, 0.3]),
                                   rtol=1e-12)
        np.testing.assert_allclose(out["depth_exp"][0], a * z, rtol=1e-12)
        np.testing.assert_allclose(out["normal"][0], [0, 0, -a], atol=1e-15)
        assert out["t_final"][0] == pytest.approx(1 - a, rel=1e-13)
        assert out["count"][0] == 1
        assert out["median_id"][0] == 0 and out["depth_med"][0] == pytest.approx(z, rel=1e-14)


def test_centre_pixel_depth_is_centre_depth():
    # Eq. 4: where (u, v) = (u_c, v_c) the depth is z_c for any plane slope.
    v = view(64, 64, 64.0)
    q = np.array([0.9, 0.3, -0.2, 0.25])
    q /= np.linalg.norm(q)
    # centre on pixel (40, 20)'s centre: x = (40.5 - 32) z / 64
    z = 2.0
    mean = [(40.5 - 32) * z / 64.0, (20.5 - 32) * z / 64.0, z]
    sc = scene_from([mean], [[0.2, 0.05, 0.01]], [q], opac=[0.9], rgb=[[0.5, 0.5, 0.5]])
    rec, _, _, outs = oracle.forward(oracle.settings(), [v], sc,
                                     pixels=[pixel_index(v, [40], [20])])
    assert abs(rec[0][0, R["p0"]]) + abs(rec[0][0, R["p1"]]) > 1e-3  # tilted plane
    zc = rec[0][0, R["z"]]
    d = zc + rec[0][0, R["p0"]] * (rec[0][0, R["uc"]] - 40.5) + rec[0][0, R["p1"]] * (
        rec[0][0, R["vc"]] - 20.5)
    assert outs[0]["depth_med"][0] == pytest.approx(d, rel=1e-12)
    assert abs(rec[0][0, R["uc"]] - 40.5) < 1e-6 and abs(rec[0][0, R["vc"]] - 20.5) < 1e-6
    assert outs[0]["depth_med"][0] == pytest.approx(zc, rel=1e-6)


def test_two_gaussians_front_to_back():
    # Eq. 3 with two splats: the nearer one is blended first regardless of
    # index order.  C = a1 c1 + (1 - a1) a2 c2.
    v = view(64, 64, 64.0)
    sc = scene_from([[0, 0, 4.0], [0, 0, 2.0]], [[0.1] * 3, [0.05] * 3], opac=[0.7, 0.6],
                    rgb=[[1, 0, 0], [0, 1, 0]])
    st = oracle.settings()
    rec, _, flags, outs = oracle.forward(st, [v], sc, pixels=[pixel_index(v, [32], [32])])
    r = rec[0]
    a = []
    for g in range(2):
        dx, dy = r[g, R["uc"]] - 32.5, r[g, R["vc"]] - 32.5
        pw = 0.5 * (r[g, R["a"]] * dx * dx + 2 * r[g, R["b"]] * dx * dy + r[g, R["c"]] * dy * dy)
        a.append(r[g, R["o"]] * np.exp(-pw))
    c_near = r[1, [R["r"], R["g"], R["bl"]]]
    c_far = r[0, [R["r"], R["g"], R["bl"]]]
    np.testing.assert_allclose(outs[0]["color"][0], a[1] * c_near + (1 - a[1]) * a[0] * c_far,
                               rtol=1e-13)
    assert outs[0]["median_id"][0] == 0 if (1 - a[1]) > 0.5 else outs[0]["median_id"][0] == 1


def _stack_scene(alphas):
    # Large isotropic splats on the optical axis at increasing depth, opacity
    # chosen so that the centre pixel sees the given alphas.
    n = len(alphas)
    means = [[0, 0, 2.0 + 0.5 * i] for i in range(n)]
    return scene_from(means, [[0.5] * 3] * n, opac=alphas, rgb=[[0.5, 0.5, 0.5]] * n)


def test_median_rule_closed_form():
    # alphas 0.3, 0.4, 0.5: incoming T = 1, 0.7, 0.42 -> the last contributor
    # with incoming T > 1/2 is the second (Sec. 1, median depth reading).
    v = view(64, 64, 64.0)
    sc = _stack_scene([0.3, 0.4, 0.5])
    st = oracle.settings(dilation=0.0)
    rec, _, _, outs = oracle.forward(st, [v], sc, pixels=[pixel_index(v, [32], [32])])
    out = outs[0]
    assert out["count"][0] == 3
    assert out["median_id"][0] == 1
    # centre pixel sits 0.5 px off the splat centre in x and y
    assert out["depth_med"][0] == pytest.approx(rec[0][1, R["z"]], rel=1e-6)
    a = []
    for g in range(3):
        r = rec[0][g]
        dx, dy = r[R["uc"]] - 32.5, r[R["vc"]] - 32.5
        pw = 0.5 * (r[R["a"]] * dx * dx + 2 * r[R["b"]] * dx * dy + r[R["c"]] * dy * dy)
        a.append(r[R["o"]] * np.exp(-pw))
    a = np.array(a)
    assert 0.29 < a[0] < 0.3 and 0.39 < a[1] < 0.4 and 0.49 < a[2] < 0.5
    assert out["t_final"][0] == pytest.approx(np.prod(1 - a), rel=1e-14)
    w = a * np.array([1.0, 1 - a[0], (1 - a[0]) * (1 - a[1])])
    assert out["alpha"][0] == pytest.approx(w.sum(), rel=1e-14)


def test_stop_rule_excludes_the_stopping_gaussian():
    # alpha 0.98 three times: T = 0.02, 4e-4, then 8e-6 < 1e-4 -> stop; the
    # third is not blended (count 2, T_final 4e-4 up to the off-centre factor).
    v = view(64, 64, 64.0)
    sc = _stack_scene([0.98, 0.98, 0.98, 0.98])
    st = oracle.settings(dilation=0.0)
    _, _, _, outs = oracle.forward(st, [v], sc, pixels=[pixel_index(v, [32], [32])])
    out = outs[0]
    assert out["count"][0] == 2
    assert out["last_id"][0] == 1
    assert 3e-4 < out["t_final"][0] < 5e-4
    assert out["alpha"][0] + out["t_final"][0] == pytest.approx(1.0, abs=1e-15)


def test_alpha_clamp():
    v = view(64, 64, 64.0)
    sc = _stack_scene([0.9999])
    _, _, _, outs = oracle.forward(oracle.settings(dilation=0.0), [v], sc,
                                   pixels=[pixel_index(v, [32], [32])])
    assert outs[0]["alpha"][0] == pytest.approx(0.99, abs=1e-15)


def test_telescoping_and_constant_features():
    # Sum of weights = 1 - T_final (Eq. 3 telescopes); with equal colours
    # C = c A + T bg; with splats on the optical axis and isotropic,
    # N = (0,0,-A); equal depths give D = z A.
    rng = np.random.default_rng(2)
    v = view(64, 64, 64.0)
    n = 40
    means = np.zeros((n, 3))
    means[:, 2] = 3.0
    sc = scene_from(means, np.full((n, 3), 0.08) * rng.uniform(0.5, 2, (n, 1)),
                    opac=rng.uniform(0.05, 0.9, n), rgb=np.tile([0.3, 0.6, 0.9], (n, 1)))
    st = oracle.settings(bg=(0.2, 0.1, 0.05))
    rec, _, _, outs = oracle.forward(st, [v], sc)
    out = outs[0]
    np.testing.assert_allclose(out["alpha"] + out["t_final"], 1.0, atol=1e-14)
    c = rec[0][0, [R["r"], R["g"], R["bl"]]]
    np.testing.assert_allclose(out["color"], out["alpha"][:, None] * c[None] +
                               out["t_final"][:, None] * np.array([0.2, 0.1, 0.05])[None],
                               atol=1e-14)
    np.testing.assert_allclose(out["normal"][:, 2], -out["alpha"], atol=1e-14)
    np.testing.assert_allclose(out["normal"][:, :2], 0.0, atol=1e-14)
    np.testing.assert_allclose(out["depth_exp"], 3.0 * out["alpha"], rtol=1e-6, atol=1e-14)


def test_mirror_symmetry():
    # Mirror x -> -x (quaternion (w,x,y,z) -> (w,x,-y,-z), degree 0) with the
    # principal point at the image centre: maps mirror, N_x flips sign.
    rng = np.random.default_rng(4)
    v = view(48, 40, 50.0)
    n = 80
    means = rng.uniform(-0.5, 0.5, (n, 3)) + np.array([0, 0, 2.5])
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    s = np.exp(rng.normal(-3, 0.5, (n, 3)))
    o = rng.uniform(0.1, 0.95, n)
    rgb = rng.uniform(0, 1, (n, 3))
    a = scene_from(means, s, q, o, rgb)
    mb = means.copy()
    mb[:, 0] *= -1
    qb = q.copy()
    qb[:, 2:] *= -1
    b = scene_from(mb, s, qb, o, rgb)
    st = oracle.settings()
    _, _, _, oa = oracle.forward(st, [v], a)
    _, _, _, ob = oracle.forward(st, [v], b)

    def img(x):
        return x.reshape(v.height, v.width, *x.shape[1:])
    np.testing.assert_allclose(img(oa[0]["color"]), img(ob[0]["color"])[:, ::-1], atol=1e-12)
    np.testing.assert_allclose(img(oa[0]["depth_exp"]), img(ob[0]["depth_exp"])[:, ::-1], atol=1e-12)
    na, nb = img(oa[0]["normal"]), img(ob[0]["normal"])[:, ::-1]
    np.testing.assert_allclose(na[..., 0], -nb[..., 0], atol=1e-12)
    np.testing.assert_allclose(na[..., 1:], nb[..., 1:], atol=1e-12)


def test_translation_invariance_with_sh():
    # Moving the world and the camera by the same translation leaves every
    # map unchanged (SH degree 3: view directions are unchanged too).
    import synth
    scene = synth.make_scene_uniform_cube(200, seed=9, sh_degree=3)
    v0 = view(48, 48, 48.0)
    shift = np.array([0.25, -0.5, 0.75], np.float32)
    moved = scene_from(scene.means + shift, scene.scales, scene.quats, scene.opacities,
                       sh=scene.sh, degree=3)
    v1 = view(48, 48, 48.0, t=-shift)
    st = oracle.settings(sh_degree=3)
    _, _, _, oa = oracle.forward(st, [v0], scene)
    _, _, _, ob = oracle.forward(st, [v1], moved)
    # the FP32 shift moves means by ~1e-7; maps agree to that level
    for k in ("color", "depth_exp", "normal", "alpha"):
        np.testing.assert_allclose(oa[0][k], ob[0][k], atol=2e-5)
