"""The oracle's hand-written adjoint against central finite differences of its
own FP64 forward (pins the adjoint; the forward is pinned elsewhere).

A perturbation is only used when it leaves every discrete decision of the
forward unchanged (contributor lists, stop and median choices, clamps, culls):
the discrete-signature guard."""
import numpy as np
import pytest

import oracle
import synth
from oracle_helpers import scene_from, view


def _loss_and_sig(st, views, scene, gouts):
    rec, rect, flags, outs = oracle.forward(st, views, scene, want_sig=True)
    L = 0.0
    sig = [flags.copy()]
    for vi, out in enumerate(outs):
        F = np.concatenate([out["color"], out["depth_exp"][:, None], out["depth_med"][:, None],
                            out["normal"], out["alpha"][:, None]], axis=1)
        L += float((F * gouts[vi]).sum())
        sig.append(out["sig"].copy())
    return L, sig


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def _scene_small(seed, degree=3, n=24):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-0.45, 0.45, (n, 3)) + np.array([0, 0, 2.2])
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    k = (degree + 1) ** 2
    sh = rng.normal(0, 0.3, (n, k, 3))
    sh[:, 0, :] += 0.8
    return scene_from(means, np.exp(rng.normal(-2.6, 0.5, (n, 3))), q,
                      rng.uniform(0.2, 0.95, n), sh=sh, degree=degree)


def _views_two():
    from scipy.spatial.transform import Rotation
    R1 = Rotation.from_rotvec([0.05, -0.08, 0.03]).as_matrix().astype(np.float32)
    return [view(20, 16, 22.0), view(18, 18, 20.0, R=R1, t=[0.05, -0.02, 0.1])]


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_matches_central_differences(seed):
    views = _views_two()
    scene = _scene_small(seed)
    st = oracle.settings(sh_degree=3, bg=(0.1, 0.3, 0.2))
    rng = np.random.default_rng(50 + seed)
    gouts = [rng.normal(size=(v.pixels, 9)) for v in views]
    grads = oracle.backward(st, views, scene, gouts)
    L0, sig0 = _loss_and_sig(st, views, scene, gouts)

    groups = ["means", "scales", "quats", "opacities", "sh"]
    checked = skipped = 0
    for grp in groups:
        arr = getattr(scene, grp)
        g = grads[grp].reshape(-1)
        scale = np.abs(g).max()
        flat_idx = rng.choice(arr.size, size=min(arr.size, 40), replace=False)
        for fi in flat_idx:
            orig = arr.reshape(-1)[fi]
            h = 3e-5 * max(abs(float(orig)), 1e-2)
            plus, minus = np.float32(orig + h), np.float32(orig - h)
            arr.reshape(-1)[fi] = plus
            Lp, sp = _loss_and_sig(st, views, scene, gouts)
            arr.reshape(-1)[fi] = minus
            Lm, sm = _loss_and_sig(st, views, scene, gouts)
            arr.reshape(-1)[fi] = orig
            if not (_same(sp, sig0) and _same(sm, sig0)):
                skipped += 1
                continue
            step = float(plus) - float(minus)
            fd = (Lp - Lm) / step
            # truncation (h^2, measured ~1e-9 relative) + FP64 round-off of L / step
            tol = 1e-6 * (abs(fd) + 1e-3 * scale) + 1e-14 * (abs(L0) + 1.0) / step
            assert abs(g[fi] - fd) <= tol, (grp, fi, g[fi], fd)
            checked += 1
    assert checked >= 150 and skipped <= 0.2 * (checked + skipped), (checked, skipped)


def test_adjoint_on_pixel_subset_equals_masked_full():
    # The VJP restricted to a pixel list equals the full VJP with zero
    # upstream gradients elsewhere (used for sampled-pixel parity at scale).
    v = view(24, 20, 24.0)
    scene = _scene_small(3, degree=1)
    st = oracle.settings(sh_degree=1)
    rng = np.random.default_rng(1)
    pix = np.sort(rng.choice(v.pixels, 60, replace=False)).astype(np.int64)
    g_sub = rng.normal(size=(60, 9))
    g_full = np.zeros((v.pixels, 9))
    g_full[pix] = g_sub
    a = oracle.backward(st, [v], scene, [g_sub], pixels=[pix])
    b = oracle.backward(st, [v], scene, [g_full])
    for k in a:
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-14)


def test_median_gradient_flows_only_to_median_splat():
    # d(median depth)/d(z of the median splat) = 1 through d = z + p.delta,
    # and zero for every other splat's depth.
    v = view(64, 64, 64.0)
    sc = scene_from([[0, 0, 2.0], [0, 0, 2.5], [0, 0, 3.0]], [[0.5] * 3] * 3,
                    opac=[0.3, 0.4, 0.5], rgb=[[0.5] * 3] * 3)
    st = oracle.settings(dilation=0.0)
    pix = np.array([32 * 64 + 32], np.int64)
    g = np.zeros((1, 9))
    g[0, 4] = 1.0
    rec, _, flags = oracle.project(st, [v], sc)
    gP = oracle.render_bwd(st, v, rec[0], flags[0], g, pix)
    zi = oracle.G_FIELDS.index("z")
    np.testing.assert_allclose(gP[:, zi], [0.0, 1.0, 0.0], atol=1e-15)


def test_workload_recipe_adjoint_fd_spot_check():
    # Same FD check on a 300-Gaussian subsample of the 800x800 recipe rendered
    # at a reduced 40x40 crop of the principal point (degree-3 SH).
    scene, _ = synth.make_workload("plain_800x800_200k", n=300)
    v = view(40, 40, 40.0)
    st = oracle.settings(sh_degree=3)
    rng = np.random.default_rng(9)
    gouts = [rng.normal(size=(v.pixels, 9))]
    grads = oracle.backward(st, [v], scene, gouts)
    L0, sig0 = _loss_and_sig(st, [v], scene, gouts)
    checked = 0
    for grp in ("means", "scales", "quats", "opacities", "sh"):
        arr = getattr(scene, grp)
        g = grads[grp].reshape(-1)
        scale = np.abs(g).max()
        nz = np.flatnonzero(g)
        for fi in rng.choice(nz, size=min(12, nz.size), replace=False):
            orig = arr.reshape(-1)[fi]
            h = 3e-5 * max(abs(float(orig)), 1e-2)
            plus, minus = np.float32(orig + h), np.float32(orig - h)
            arr.reshape(-1)[fi] = plus
            Lp, sp = _loss_and_sig(st, [v], scene, gouts)
            arr.reshape(-1)[fi] = minus
            Lm, sm = _loss_and_sig(st, [v], scene, gouts)
            arr.reshape(-1)[fi] = orig
            if not (_same(sp, sig0) and _same(sm, sig0)):
                continue
            step = float(plus) - float(minus)
            fd = (Lp - Lm) / step
            tol = 1e-6 * (abs(fd) + 1e-3 * scale) + 1e-14 * (abs(L0) + 1.0) / step
            assert abs(g[fi] - fd) <= tol, (grp, fi)
            checked += 1
    assert checked >= 40
