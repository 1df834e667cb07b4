"""Pins of the oracle's depth-distortion term (Sec. 3.4, Eq. 23):
sum over ordered pairs of blended splats of w_i w_j (d_i - d_j)^2, with the
blend weights held constant in its adjoint (the training loss detaches them,
Sec. 4.1)."""
import numpy as np

import oracle
from oracle_helpers import pixel_index, scene_from, view

R = oracle.R


def _alphas_at(rec, px, py):
    a = []
    for g in range(rec.shape[0]):
        dx, dy = rec[g, R["uc"]] - (px + 0.5), rec[g, R["vc"]] - (py + 0.5)
        pw = 0.5 * (rec[g, R["a"]] * dx * dx + 2 * rec[g, R["b"]] * dx * dy +
                    rec[g, R["c"]] * dy * dy)
        a.append(min(0.99, rec[g, R["o"]] * np.exp(-pw)))
    return np.array(a)


def test_two_splats_closed_form():
    # Two isotropic splats on the optical axis: depth planes are flat (q = 0),
    # so d_i = z_i at every pixel; w_near = a_near, w_far = (1 - a_near) a_far
    # and the double sum is 2 w_near w_far (z_far - z_near)^2.
    v = view(64, 64, 64.0)
    sc = scene_from([[0, 0, 4.0], [0, 0, 2.5]], [[0.2] * 3, [0.15] * 3], opac=[0.7, 0.6])
    st = oracle.settings()
    pix = [pixel_index(v, [32, 30, 35], [32, 33, 29])]
    rec, _, flags, outs = oracle.forward(st, [v], sc, pixels=pix)
    r = rec[0]
    for k, (px, py) in enumerate([(32, 32), (30, 33), (35, 29)]):
        a = _alphas_at(r, px, py)
        w_near, w_far = a[1], (1 - a[1]) * a[0]
        z_near, z_far = r[1, R["z"]], r[0, R["z"]]
        ref = 2 * w_near * w_far * (z_far - z_near) ** 2
        np.testing.assert_allclose(outs[0]["distortion"][k], ref, rtol=1e-12)
        assert outs[0]["count"][k] == 2


def test_zero_for_one_splat_and_for_equal_depths():
    v = view(48, 48, 48.0)
    one = scene_from([[0.1, 0, 3.0]], [[0.3] * 3], opac=[0.8])
    st = oracle.settings()
    _, _, _, outs = oracle.forward(st, [v], one)
    assert np.all(outs[0]["distortion"] == 0.0)
    # three isotropic splats at the same depth (d_i equal at every pixel)
    flat = scene_from([[0, 0, 3.0], [0.05, 0, 3.0], [0, 0.05, 3.0]], [[0.2] * 3] * 3,
                      opac=[0.5, 0.4, 0.3])
    _, _, _, outs = oracle.forward(st, [v], flat)
    assert outs[0]["count"].max() == 3
    assert np.abs(outs[0]["distortion"]).max() < 1e-20


def test_equals_weighted_variance_identity():
    # sum_{i,j} w_i w_j (d_i - d_j)^2 = 2 (A sum_i w_i d_i^2 - (sum_i w_i d_i)^2)
    # checked per pixel on a random scene from the blended list the oracle
    # exposes through its expected depth and alpha, with the second moment
    # recomputed from the same weights.
    rng = np.random.default_rng(3)
    n = 60
    means = rng.uniform(-0.5, 0.5, (n, 3)) + np.array([0, 0, 3.0])
    q = rng.normal(size=(n, 4))
    sc = scene_from(means, np.exp(rng.normal(-2.2, 0.4, (n, 3))), q / np.linalg.norm(q, axis=1)[:, None],
                    rng.uniform(0.2, 0.9, n))
    v = view(40, 40, 40.0)
    st = oracle.settings()
    rec, _, flags, outs = oracle.forward(st, [v], sc)
    out = outs[0]
    r = rec[0]
    order = np.lexsort((np.arange(n), r[:, R["z"]].astype(np.float32)))
    vis = (flags[0] & oracle.F_VISIBLE) != 0
    checked = 0
    for p in rng.choice(v.pixels, 400, replace=False):
        px, py = p % v.width, p // v.width
        T, ws, ds = 1.0, [], []
        for g in order:
            if not vis[g]:
                continue
            dx, dy = r[g, R["uc"]] - (px + 0.5), r[g, R["vc"]] - (py + 0.5)
            pw = 0.5 * (r[g, R["a"]] * dx * dx + 2 * r[g, R["b"]] * dx * dy + r[g, R["c"]] * dy * dy)
            if pw > 4.5:
                continue
            a = min(0.99, r[g, R["o"]] * np.exp(-pw))
            if a < 1 / 255:
                continue
            if T * (1 - a) < 1e-4:
                break
            ws.append(a * T)
            ds.append(r[g, R["z"]] + r[g, R["p0"]] * dx + r[g, R["p1"]] * dy)
            T *= 1 - a
        ws, ds = np.array(ws), np.array(ds)
        if ws.size < 2:
            continue
        A, D1, D2 = ws.sum(), (ws * ds).sum(), (ws * ds * ds).sum()
        np.testing.assert_allclose(out["alpha"][p], A, rtol=1e-12)
        np.testing.assert_allclose(out["depth_exp"][p], D1, rtol=1e-12)
        np.testing.assert_allclose(out["distortion"][p], 2 * (A * D2 - D1 * D1), rtol=1e-8,
                                   atol=1e-12 * D2 * A)
        checked += 1
    assert checked > 50


def test_adjoint_matches_central_differences_of_depth_fields():
    # The weights do not depend on a splat's depth plane (z, p): perturbing
    # those record fields changes only the d_i, so central differences of the
    # distortion there equal the detached-weight adjoint.  z is perturbed
    # less than any gap between depths, so the blend order is unchanged.
    rng = np.random.default_rng(7)
    n = 12
    means = rng.uniform(-0.3, 0.3, (n, 3)) + np.array([0, 0, 2.5])
    q = rng.normal(size=(n, 4))
    sc = scene_from(means, np.exp(rng.normal(-2.0, 0.3, (n, 3))), q / np.linalg.norm(q, axis=1)[:, None],
                    rng.uniform(0.3, 0.8, n))
    v = view(24, 24, 24.0)
    st = oracle.settings()
    rec, _, flags = oracle.project(st, [v], sc)
    r = rec[0].copy()
    g = rng.normal(size=v.pixels)
    gout = np.zeros((v.pixels, 10))
    gout[:, 9] = g
    gP = oracle.render_bwd(st, v, r, flags[0], gout)

    def loss(rr):
        return float((oracle.render(st, v, rr, flags[0])["distortion"] * g).sum())

    G = {f: i for i, f in enumerate(oracle.G_FIELDS)}
    checked = 0
    for gi in range(n):
        if not (flags[0][gi] & oracle.F_VISIBLE):
            continue
        for field in ("z", "p0", "p1"):
            h = 1e-6 * max(1.0, abs(r[gi, R[field]]))
            rp, rm = r.copy(), r.copy()
            rp[gi, R[field]] += h
            rm[gi, R[field]] -= h
            fd = (loss(rp) - loss(rm)) / (2 * h)
            ad = gP[gi, G[field]]
            assert abs(fd - ad) <= 1e-6 * (abs(ad) + 1e-3 * np.abs(gP[:, G[field]]).max()), \
                (gi, field, fd, ad)
            checked += 1
    assert checked >= 15
