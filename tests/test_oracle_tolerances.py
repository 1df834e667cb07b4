"""Pins of the oracle's tolerance machinery: the quantities that set the
floors and exclusions of every GPU parity comparison.

* gradient_error_scale S (the round-off scale of a gradient element: the
  adjoint of Eq. 3 run on magnitudes, pushed through |d parameter / d splat
  quantity|): a bound of the gradient and of every per-pixel contribution to
  it, equal to |g| where the gradient is one term, additive over pixels and
  homogeneous in the upstream gradient.
* dist_mag (the round-off scale of the depth distortion of Eq. 23): the
  first-order change of the distortion under relative depth perturbations of
  size eps is at most 2 eps dist_mag, attained with two splats.
* the magnitude bound of the Eq. 24 median-depth gradient: at least the sum
  over interior pixels q of |d L_q / d D(p)| (by central differences of each
  pixel's own term), hence at least |d L / d D(p)|.
* the fragile-pixel flags: set exactly when a splat of the pixel lies within
  the stated margin of a discrete threshold of Eq. 3 (3-sigma cut, alpha_min,
  t_min stop, the median's T = 1/2, the alpha_max clamp); pixels without a
  flag keep every discrete decision when the splat records are rounded to
  FP32 and perturbed by a few units in the last place.
"""
import numpy as np
import pytest

import oracle
from oracle_helpers import pixel_index, scene_from, view

R = oracle.R
G = {k: i for i, k in enumerate(oracle.G_FIELDS)}


def _scene(seed, n=24, degree=3):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-0.45, 0.45, (n, 3)) + np.array([0, 0, 2.2])
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    k = (degree + 1) ** 2
    sh = rng.normal(0, 0.3, (n, k, 3))
    sh[:, 0, :] += 0.8
    return scene_from(means, np.exp(rng.normal(-2.6, 0.5, (n, 3))), q,
                      rng.uniform(0.2, 0.95, n), sh=sh, degree=degree)


def _views():
    from scipy.spatial.transform import Rotation
    R1 = Rotation.from_rotvec([0.05, -0.08, 0.03]).as_matrix().astype(np.float32)
    return [view(20, 16, 22.0), view(18, 18, 20.0, R=R1, t=[0.05, -0.02, 0.1])]


# ---------------------------------------------------------------------------
# gradient_error_scale

def test_scale_bounds_the_gradient_and_every_pixel_contribution():
    """S >= sum over pixels of |that pixel's contribution| >= |g|, per
    element of every parameter group; the per-pixel contributions come from
    separate one-pixel VJPs (another route through the adjoint)."""
    views = _views()
    scene = _scene(0)
    st = oracle.settings(sh_degree=3, bg=(0.1, 0.3, 0.2))
    rng = np.random.default_rng(7)
    pix = [np.sort(rng.choice(v.pixels, 40, replace=False)).astype(np.int64) for v in views]
    gouts = [rng.normal(size=(len(p), 9)) for p in pix]
    g = oracle.backward(st, views, scene, gouts, pixels=pix)
    S = oracle.gradient_error_scale(st, views, scene, gouts, pixels=pix)
    per_pixel = {k: np.zeros_like(a) for k, a in g.items()}
    empty = np.zeros(0, np.int64)
    for vi in range(len(views)):
        for j in range(len(pix[vi])):
            pl = [empty] * len(views)
            go = [np.zeros((0, 9))] * len(views)
            pl[vi] = pix[vi][j:j + 1]
            go[vi] = gouts[vi][j:j + 1]
            gj = oracle.backward(st, views, scene, go, pixels=pl)
            for k in gj:
                per_pixel[k] += np.abs(gj[k])
    nontrivial = 0
    for k in g:
        a, b, s = np.abs(g[k]), per_pixel[k], S[k]
        assert (a <= b * (1 + 1e-12) + 1e-300).all(), k
        assert (b <= s * (1 + 1e-9) + 1e-300).all(), k
        nontrivial += int((b > 0).sum())
    assert nontrivial > 500


def test_scale_equals_the_gradient_when_it_is_one_term():
    """One Gaussian, one pixel, bg = 0.  With upstream gradient on colour
    channel 0 only, the SH DC coefficient of channel 0 receives w Y00 g (one
    term); with upstream gradient on alpha only, the opacity receives e^-power
    g (one term, T = 1, nothing behind).  S equals |g| there."""
    v = view(32, 32, 32.0)
    sc = scene_from([[0.02, -0.01, 3.0]], [[0.08] * 3], opac=[0.6], rgb=[[0.7, 0.2, 0.4]])
    st = oracle.settings()
    pix = [np.array([pixel_index(v, 16, 16)], np.int64)]
    for col, grp, idx in ((0, "sh", (0, 0)), (8, "opacities", (0,))):
        go = np.zeros((1, 9))
        go[0, col] = -1.7
        g = oracle.backward(st, [v], sc, [go], pixels=pix)
        S = oracle.gradient_error_scale(st, [v], sc, [go], pixels=pix)
        gv = np.asarray(g[grp]).reshape(g[grp].shape[0], -1)[idx[0], idx[1] if len(idx) > 1 else 0] \
            if g[grp].ndim > 1 else g[grp][idx[0]]
        sv = np.asarray(S[grp]).reshape(S[grp].shape[0], -1)[idx[0], idx[1] if len(idx) > 1 else 0] \
            if S[grp].ndim > 1 else S[grp][idx[0]]
        assert gv != 0.0
        assert sv == pytest.approx(abs(gv), rel=1e-12), (grp, gv, sv)


def test_scale_is_additive_over_pixels_and_homogeneous():
    views = _views()[:1]
    scene = _scene(1)
    st = oracle.settings(sh_degree=3)
    rng = np.random.default_rng(3)
    v = views[0]
    allp = rng.permutation(v.pixels).astype(np.int64)
    p1, p2 = np.sort(allp[:60]), np.sort(allp[60:130])
    g1, g2 = rng.normal(size=(60, 9)), rng.normal(size=(70, 9))
    S1 = oracle.gradient_error_scale(st, views, scene, [g1], pixels=[p1])
    S2 = oracle.gradient_error_scale(st, views, scene, [g2], pixels=[p2])
    p12 = np.concatenate([p1, p2])
    S12 = oracle.gradient_error_scale(st, views, scene, [np.concatenate([g1, g2])],
                                      pixels=[p12])
    S1n = oracle.gradient_error_scale(st, views, scene, [-3.0 * g1], pixels=[p1])
    for k in S1:
        np.testing.assert_allclose(S12[k], S1[k] + S2[k], rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(S1n[k], 3.0 * S1[k], rtol=1e-12, atol=1e-300)
        assert (S1[k] >= 0).all()


# ---------------------------------------------------------------------------
# dist_mag of Eq. 23

def _depth_scene():
    # isotropic splats at well separated depths over the image centre: their
    # blend order and alphas do not depend on small changes of the depth
    # fields, whose planes are flat (q = 0)
    return scene_from([[0.0, 0.0, 2.0], [0.01, 0.005, 2.6], [-0.01, 0.0, 3.3],
                       [0.0, -0.01, 4.1]], [[0.05] * 3, [0.07] * 3, [0.09] * 3, [0.12] * 3],
                      opac=[0.35, 0.5, 0.45, 0.7])


def _perturbed(rec, eps):
    r = rec.copy()
    for k in ("z", "p0", "p1"):
        r[:, R[k]] *= 1.0 + eps
    return r


def test_distortion_magnitude_bounds_first_order_change():
    """Depths scaled by (1 + eps_i) with |eps_i| <= eps (z and the plane p
    scaled together scale every per-pixel depth d = z + p . delta): the
    distortion changes by at most 2 eps dist_mag (to first order, eps =
    1e-7), on pixels with 2 to 4 blended splats."""
    v = view(32, 32, 32.0)
    sc = _depth_scene()
    st = oracle.settings()
    rec, _, flags = oracle.project(st, [v], sc)
    rec, flags = rec[0], flags[0]
    base = oracle.render(st, v, rec, flags)
    rng = np.random.default_rng(11)
    eps = 1e-7
    use = base["count"] >= 2
    assert use.sum() > 20 and base["count"].max() >= 3
    worst = 0.0
    for _ in range(20):
        e = rng.uniform(-eps, eps, rec.shape[0])
        out = oracle.render(st, v, _perturbed(rec, e), flags)
        assert np.array_equal(out["count"], base["count"])
        d = np.abs(out["distortion"] - base["distortion"])[use]
        bound = 2 * eps * base["distortion_mag"][use]
        assert (d <= bound * (1 + 1e-5) + 1e-30).all()
        worst = max(worst, float((d / bound).max()))
    assert worst > 0.05  # the bound is not vacuous


def test_distortion_magnitude_attained_by_two_splats():
    """With two blended splats the worst relative perturbation (eps_i =
    eps sign of d dist / d d_i, i.e. moving the depths apart) changes the
    distortion by 2 eps dist_mag to first order."""
    v = view(32, 32, 32.0)
    sc = scene_from([[0.0, 0.0, 2.0], [0.0, 0.0, 3.0]], [[0.1] * 3, [0.1] * 3], opac=[0.5, 0.6])
    st = oracle.settings()
    rec, _, flags = oracle.project(st, [v], sc)
    rec, flags = rec[0], flags[0]
    pix = np.array([pixel_index(v, 16, 16), pixel_index(v, 17, 15)], np.int64)
    base = oracle.render(st, v, rec, flags, pix)
    assert (base["count"] == 2).all()
    eps = 1e-8
    # the nearer splat moves nearer, the farther one farther
    e = np.array([-eps, eps])
    out = oracle.render(st, v, _perturbed(rec, e), flags, pix)
    ratio = (out["distortion"] - base["distortion"]) / (2 * eps * base["distortion_mag"])
    np.testing.assert_allclose(ratio, 1.0, rtol=1e-6)


# ---------------------------------------------------------------------------
# Eq. 24 median-depth gradient magnitude

def _nc_maps(seed, H=9, W=11):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    D = 3.0 + 0.05 * xx + 0.08 * yy + 0.03 * np.sin(xx + 2 * yy) + 0.02 * rng.normal(size=(H, W))
    N = rng.normal(size=(3, H, W)) * 0.3
    N[2] -= 0.6
    A = rng.uniform(0.2, 1.0, size=(H, W))
    return D, N, A


@pytest.mark.parametrize("seed", [0, 1])
def test_nc_depth_magnitude_bounds_every_pixel_term(seed):
    """gD_mag(p) >= sum_q |d L_q / d D(p)| >= |d L / d D(p)|, where L_q is
    pixel q's own term of Eq. 24 (isolated by zeroing the normal and alpha
    maps elsewhere: n~ depends on the depths only) and its derivative is a
    central difference.  Scaling the weight scales the bound."""
    v = view(11, 9, 10.0)
    D, N, A = _nc_maps(seed)
    H, W = D.shape
    w = 5.0
    _, gD, _, _, gD_mag = oracle.normal_consistency(v, D, N, A, w, magnitude=True)
    terms = np.zeros((H, W))
    for qy in range(1, H - 1):
        for qx in range(1, W - 1):
            Nq = np.zeros_like(N)
            Aq = np.zeros_like(A)
            Nq[:, qy, qx] = N[:, qy, qx]
            Aq[qy, qx] = A[qy, qx]
            for py, px in ((qy, qx - 1), (qy, qx + 1), (qy - 1, qx), (qy + 1, qx), (qy, qx)):
                h = 1e-6 * abs(D[py, px])
                o = D[py, px]
                D[py, px] = o + h
                lp = oracle.normal_consistency(v, D, Nq, Aq, w)[0]
                D[py, px] = o - h
                lm = oracle.normal_consistency(v, D, Nq, Aq, w)[0]
                D[py, px] = o
                terms[py, px] += abs((lp - lm) / (2 * h))
    assert (np.abs(gD) <= terms * (1 + 1e-5) + 1e-12).all()
    assert (terms <= gD_mag * (1 + 1e-5) + 1e-12).all()
    assert (terms > 0).sum() > 0.8 * H * W - 4
    _, _, _, _, gD_mag2 = oracle.normal_consistency(v, D, -N, A, -2.0 * w, magnitude=True)
    np.testing.assert_allclose(gD_mag2, 2.0 * gD_mag, rtol=1e-12)


# ---------------------------------------------------------------------------
# fragile-pixel flags

def _record(uc, vc, conic, o, z, rgb=(0.5, 0.5, 0.5)):
    r = np.zeros(len(oracle.R_FIELDS))
    r[R["uc"]], r[R["vc"]] = uc, vc
    r[R["a"]], r[R["b"]], r[R["c"]] = conic
    r[R["o"]], r[R["z"]] = o, z
    r[R["r"]], r[R["g"]], r[R["bl"]] = rgb
    r[R["n2"]] = -1.0
    return r


def _render_records(recs, st=None, px=0, py=0):
    st = oracle.settings() if st is None else st
    v = view(4, 4, 4.0)
    rec = np.stack(recs)
    flags = np.full(rec.shape[0], oracle.F_VISIBLE, np.int32)
    return oracle.render(st, v, rec, flags, np.array([pixel_index(v, px, py)], np.int64),
                         want_sig=True)


def _at_power(p, o=0.5, z=2.0):
    # isotropic conic a = c = 1: power = dx^2 / 2 with dx = u_c - 0.5
    return _record(0.5 + np.sqrt(2.0 * p), 0.5, (1.0, 0.0, 1.0), o, z)


@pytest.mark.parametrize("delta,flagged", [(1e-5, True), (-1e-5, True), (5e-5, False),
                                           (-5e-5, False)])
def test_flag_power_cut(delta, flagged):
    out = _render_records([_at_power(4.5 + delta, o=0.9)])
    assert bool(out["fragile"][0] & 1) == flagged


@pytest.mark.parametrize("rel,flagged", [(5e-6, True), (-5e-6, True), (3e-5, False),
                                         (-3e-5, False)])
def test_flag_alpha_min(rel, flagged):
    # power 1, alpha = o e^-1 placed relative to alpha_min = 1/255
    o = (1.0 / 255.0) * (1.0 + rel) * np.e
    out = _render_records([_at_power(1.0, o=o)])
    assert bool(out["fragile"][0] & 1) == flagged
    assert out["count"][0] == (1 if rel > 0 else 0)


@pytest.mark.parametrize("rel,flagged", [(5e-5, True), (-5e-5, True), (3e-4, False),
                                         (-3e-4, False)])
def test_flag_transmittance_stop(rel, flagged):
    # two splats at the pixel centre (power 0): T' = (1 - a1)(1 - a2) placed
    # relative to t_min = 1e-4
    a1 = 0.99
    a2 = 1.0 - 1e-4 * (1.0 + rel) / (1.0 - a1)
    st = oracle.settings(alpha_max=0.999999)
    out = _render_records([_record(0.5, 0.5, (1, 0, 1), a1, 2.0),
                           _record(0.5, 0.5, (1, 0, 1), a2, 3.0)], st)
    assert bool(out["fragile"][0] & 1) == flagged
    assert out["count"][0] == (2 if rel > 0 else 1)


@pytest.mark.parametrize("rel,flagged", [(4e-6, True), (-4e-6, True), (4e-5, False),
                                         (-4e-5, False)])
def test_flag_median_half(rel, flagged):
    # T before the second splat = 1 - a1, placed relative to 1/2
    a1 = 1.0 - 0.5 * (1.0 + rel)
    out = _render_records([_record(0.5, 0.5, (1, 0, 1), a1, 2.0),
                           _record(0.5, 0.5, (1, 0, 1), 0.3, 3.0)])
    assert bool(out["fragile"][0] & 1) == flagged
    assert out["median_id"][0] == (1 if rel > 0 else 0)


@pytest.mark.parametrize("rel,flagged", [(5e-6, True), (-5e-6, True), (3e-5, False),
                                         (-3e-5, False)])
def test_flag_alpha_clamp_is_a_gradient_flag(rel, flagged):
    # raw alpha = o at the centre, placed relative to alpha_max = 0.99: the
    # clamp changes the gradient (d alpha = 0), not the maps: bit 1 only
    out = _render_records([_record(0.5, 0.5, (1, 0, 1), 0.99 * (1.0 + rel), 2.0)])
    assert bool(out["fragile"][0] & 2) == flagged
    assert not out["fragile"][0] & 1


def test_unflagged_pixels_keep_their_decisions_under_fp32_rounding():
    """A dense random scene: every pixel with no fragile flag keeps its
    discrete signature (contributors in order, clamps, median, stop) when
    every record field is rounded to FP32 and then perturbed by up to 4
    units in the last place -- the rounding the GPU path applies to the
    splats; flagged pixels are few."""
    rng = np.random.default_rng(21)
    n = 400
    means = rng.uniform(-0.5, 0.5, (n, 3)) + np.array([0, 0, 2.5])
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    sc = scene_from(means, np.exp(rng.normal(-2.8, 0.5, (n, 3))), q, opac=rng.uniform(0.05, 1, n))
    v = view(48, 40, 48.0)
    st = oracle.settings()
    rec, _, flags = oracle.project(st, [v], sc)
    rec, flags = rec[0], flags[0]
    base = oracle.render(st, v, rec, flags, want_sig=True)
    stable = base["fragile"] == 0
    assert stable.mean() > 0.97
    changed_stable = 0
    flips = 0
    for trial in range(4):
        r32 = rec.astype(np.float32).astype(np.float64)
        ulp = np.spacing(np.abs(rec).astype(np.float32)).astype(np.float64)
        r32 += rng.integers(-4, 5, rec.shape) * ulp
        r32[:, R["z"]] = rec[:, R["z"]]  # the blend order is by float32(z) on both sides
        out = oracle.render(st, v, r32, flags, want_sig=True)
        diff = out["sig"] != base["sig"]
        changed_stable += int((diff & stable).sum())
        flips += int(diff.sum())
    assert changed_stable == 0, changed_stable
