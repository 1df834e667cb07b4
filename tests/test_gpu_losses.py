"""GPU parity of the fused normal-consistency regulariser (Eq. 24) with the
FP64 oracle, on rendered maps and on a smooth synthetic surface, several
views packed back to back."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import device, gpu_forward, say

pytestmark = pytest.mark.gpu


def _check(got, ref, what, tol=1e-4, mag=None):
    """|g - g_ref| <= tol (|g_ref| + 1e-3 max|g_ref| [+ 0.1 mag]); mag is the
    oracle's round-off scale of the depth gradient (a discrete divergence of
    per-pixel terms that cancel on smooth maps)."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    floor = 1e-3 * np.abs(ref).max() + 1e-30
    if mag is not None:
        floor = floor + 0.1 * np.asarray(mag, np.float64)
    err = np.abs(got - ref) / (np.abs(ref) + floor)
    say(f"  {what}: worst {err.max():.3g}")
    assert err.max() <= tol, (what, err.max())


def _run(views, depth, normal, alpha, weight, dev):
    """Run the kernel twice: onto zero gradient maps (the values compared with
    the oracle) and onto random ones, which must receive exactly the same
    additions (one FP32 add per element)."""
    import torch
    from paper_2406_01467_amd import _lib
    vc = _lib.make_views(views)
    P, _ = _lib.rade_views_prepare(_lib.Settings(), vc)
    vdev = _lib.views_to_device(vc, dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    D, N, A = t(depth), t(normal), t(alpha)
    ws = torch.empty(_lib.rade_normal_consistency_workspace(P), dtype=torch.uint8, device=dev)
    rng = np.random.default_rng(0)
    outs = []
    for base in ([np.zeros(k * P, np.float32) for k in (2, 3, 1)],
                 [rng.normal(size=k * P).astype(np.float32) for k in (2, 3, 1)]):
        loss = torch.zeros(len(views), device=dev)
        gD, gN, gA = (t(b) for b in base)
        _lib.rade_normal_consistency(vc, vdev, D, N, A, weight, loss, gD, gN, gA, ws)
        torch.cuda.synchronize()
        outs.append((loss.cpu().numpy(), [x.cpu().numpy() for x in (gD, gN, gA)], base))
    (l0, g0, _), (l1, g1, b1) = outs
    np.testing.assert_allclose(l1, l0, rtol=1e-6)  # order of the FP32 atomic adds may differ
    for a, b, z in zip(g0, g1, b1):
        assert np.array_equal(b, (z + a).astype(np.float32))  # accumulated, not overwritten
    # overwrite mode: whatever the maps held (NaN here), the result has the
    # bits of the accumulation into zeroed maps
    loss = torch.zeros(len(views), device=dev)
    gD, gN, gA = (torch.full((k * P,), float("nan"), device=dev) for k in (2, 3, 1))
    _lib.rade_normal_consistency(vc, vdev, D, N, A, weight, loss, gD, gN, gA, ws,
                                 accumulate=False)
    torch.cuda.synchronize()
    for a, b in zip(g0, (gD, gN, gA)):
        assert np.array_equal(a.view(np.uint32), b.cpu().numpy().view(np.uint32))
    return l0, g0[0], g0[1], g0[2], vc


def test_normal_consistency_on_rendered_maps():
    from paper_2406_01467_amd import Settings
    dev = device()
    scene = synth.make_scene_clusters(6000, seed=17, width=96, height=72, dist_range=(2, 6))
    views = [synth.identity_view(96, 72)] + synth.make_views_orbit(
        scene.means.mean(0), 5.0, 1, seed=18, sizes=[(57, 80)])
    rast, maps, gv, _ = gpu_forward(scene, views, Settings(sh_degree=3), dev)
    depth = maps.depth.cpu().numpy()
    normal = maps.normal.cpu().numpy()
    alpha = maps.alpha.cpu().numpy()
    loss, gD, gN, gA, vc = _run(views, depth, normal, alpha, 5.0, dev)
    for vi, v in enumerate(views):
        o, H, W = vc[vi].pix_offset, v.height, v.width
        P = H * W
        Dm = depth[2 * o + P: 2 * o + 2 * P].reshape(H, W)
        Nm = normal[3 * o: 3 * o + 3 * P].reshape(3, H, W)
        Am = alpha[o: o + P].reshape(H, W)
        l, rD, rN, rA, mD = oracle.normal_consistency(v, Dm, Nm, Am, 5.0, magnitude=True)
        say("view", vi, "loss", loss[vi], "ref", l)
        assert loss[vi] == pytest.approx(l, rel=1e-5)
        _check(gD[2 * o + P: 2 * o + 2 * P].reshape(H, W), rD, "d depth_med", mag=mD)
        assert np.all(gD[2 * o: 2 * o + P] == 0)  # expected-depth plane untouched
        _check(gN[3 * o: 3 * o + 3 * P].reshape(3, H, W), rN, "d normal")
        _check(gA[o: o + P].reshape(H, W), rA, "d alpha")


def test_normal_consistency_smooth_surface():
    dev = device()
    H, W = 50, 70
    v = synth.identity_view(W, H)
    yy, xx = np.mgrid[0:H, 0:W]
    D = 4.0 + 0.02 * xx - 0.015 * yy + 0.3 * np.sin(0.1 * xx) * np.cos(0.13 * yy)
    rng = np.random.default_rng(2)
    N = rng.normal(size=(3, H, W)) * 0.2
    N[2] -= 0.7
    A = rng.uniform(0.5, 1.0, size=(H, W))
    depth = np.concatenate([np.zeros(H * W), D.reshape(-1)]).astype(np.float32)
    loss, gD, gN, gA, _ = _run([v], depth, N.reshape(-1), A.reshape(-1), 2.0, dev)
    l, rD, rN, rA, mD = oracle.normal_consistency(
        v, depth[H * W:].reshape(H, W).astype(np.float64), N.astype(np.float32),
        A.astype(np.float32), 2.0, magnitude=True)
    assert loss[0] == pytest.approx(l, rel=1e-5)
    _check(gD[H * W:].reshape(H, W), rD, "d depth_med", mag=mD)
    _check(gN.reshape(3, H, W), rN, "d normal")
    _check(gA.reshape(H, W), rA, "d alpha")


def test_l1_color_gradient_matches_its_definition():
    """weight sign(C - T) / (3 W H) per view, written over every pixel
    (NaN-filled output), bit for bit the torch expression of the same
    definition; ties give 0."""
    import torch
    from paper_2406_01467_amd import _lib
    dev = device()
    views = [synth.identity_view(37, 23), synth.identity_view(64, 48), synth.identity_view(5, 7)]
    vc = _lib.make_views(views)
    P, _ = _lib.rade_views_prepare(_lib.Settings(), vc)
    vdev = _lib.views_to_device(vc, dev)
    rng = np.random.default_rng(19)
    C = rng.uniform(0, 1, 3 * P).astype(np.float32)
    T = rng.uniform(0, 1, 3 * P).astype(np.float32)
    T[::5] = C[::5]  # ties
    Cd, Td = torch.from_numpy(C).to(dev), torch.from_numpy(T).to(dev)
    for weight in (1.0, 0.37):
        out = torch.full((3 * P,), float("nan"), device=dev)
        _lib.rade_l1_color_grad(vc, vdev, Cd, Td, weight, out)
        torch.cuda.synchronize()
        want = np.zeros(3 * P, np.float32)
        for v in vc:
            n = v.width * v.height
            sl = slice(3 * v.pix_offset, 3 * v.pix_offset + 3 * n)
            w = np.float32(float(np.float32(weight)) / (3.0 * n))
            want[sl] = np.sign(C[sl] - T[sl]).astype(np.float32) * w
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), weight
        assert (got == 0).sum() >= 3 * P // 5
