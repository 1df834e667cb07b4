"""Adjoint with recomputation on the 3M-Gaussian / 32-view workload (cluster
recipe, SH degree 3, 32 orbit views of 1600x1064).  The forward saves only
the final transmittance, the last blended position and the median id per
pixel; the backward re-projects the splats from the parameters.

- at full scale: recompute and stored-splat backward agree (maps bitwise,
  gradients up to the order of FP32 atomic additions), and sampled pixels of
  the maps match the oracle (brute force over all 3M Gaussians);
- on a 2k-Gaussian subsample seen by all 32 views: the recompute gradients
  match the oracle's FP64 adjoint (the bar of the other backward tests) and
  FP64 central finite differences of the oracle forward for every parameter
  group of the Gaussians with the largest footprints.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import (compare_maps, device, grad_check, oracle_settings, say, to_dev)

pytestmark = pytest.mark.gpu

WORKLOAD = "recompute_32views_3m"


def _settings(**kw):
    from paper_2406_01467_amd import Settings
    return Settings(**kw)


def test_recompute_at_full_scale_matches_stored_splats():
    import torch
    from paper_2406_01467_amd.batched import BatchedPlan
    dev = device()
    scene, views = synth.make_workload(WORKLOAD)
    say("recompute at scale:", scene.n, "Gaussians,", len(views), "views")
    params = to_dev(scene, dev)
    s = _settings(sh_degree=3)
    gen = torch.Generator(device=dev)
    ups = {}

    def fixed(maps):
        # one set of random upstream gradients, drawn on the device
        if not ups:
            gen.manual_seed(77)
            for k, c in (("c", 3), ("d", 2), ("n", 3), ("a", 1)):
                P = maps["alpha"].numel()
                ups[k] = torch.randn(c * P, generator=gen, device=dev)
        return ups["c"], ups["d"], ups["n"], ups["a"]

    out = {}
    peak = {}
    for recompute in (False, True):
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        plan = BatchedPlan(views, s, params, fixed, recompute=recompute)
        torch.cuda.synchronize()
        # the steady state of a training loop: the plan's buffers and the
        # peak of a step (the construction's one-off sizing pass excluded)
        torch.cuda.reset_peak_memory_stats()
        n = plan.step()
        torch.cuda.synchronize()
        peak[recompute] = torch.cuda.max_memory_allocated() - base
        assert not plan.overflowed()
        say("  recompute", recompute, "pairs", plan.n_pairs(), "replays", n,
            f"peak memory {peak[recompute] / 2**30:.2f} GiB")
        out[recompute] = ({k: v.clone() for k, v in plan.maps.items()},
                          [g.clone() for g in plan.grads], plan.rast)
        del plan
    # recompute mode keeps no second copy of the V x N splat records (80 B)
    # and tile counts (4 B): the forward writes them into the region the
    # backward recomputes them in, so it needs no more memory than stored
    # mode (it needed V x N x 84 B more when the plan kept both); in both
    # modes the binning workspace and the gradient records share memory
    VN = len(views) * scene.n
    say(f"  step peak: stored {peak[False] / 2**30:.2f} GiB, recompute {peak[True] / 2**30:.2f} "
        f"GiB (splat records and counts {VN * 84 / 2**30:.2f} GiB)")
    assert peak[True] <= peak[False] + 0.02 * VN * 84
    (m0, g0, rast), (m1, g1, _) = out[False], out[True]
    for k in m0:
        assert torch.equal(m0[k], m1[k]), k
    # gradients are sums of FP32 atomic additions whose order varies from
    # run to run: same bar as the norm-wise parity with the oracle
    for a, b in zip(g0, g1):
        rel = float(torch.linalg.norm(a - b) / torch.linalg.norm(a))
        say("  recompute vs stored, relative norm of the difference", rel)
        assert rel <= 1e-5
    assert all(torch.linalg.norm(a) > 0 for a in g0)

    # sampled pixels of two views against the oracle over all 3M Gaussians
    st = oracle_settings(s)
    rng = np.random.default_rng(5)
    frag = 0
    for vi in (0, 17):
        v = views[vi]
        vc = rast.views_c[vi]
        pix = np.sort(rng.choice(v.pixels, 48, replace=False)).astype(np.int64)
        rec, _, flags = oracle.project(st, [v], scene)
        ref = oracle.render(st, v, rec[0], flags[0], pix)
        o, P = vc.pix_offset, v.pixels
        g = {
            "color": m0["color"][3 * o: 3 * (o + P)].view(3, P).cpu().numpy(),
            "depth": m0["depth"][2 * o: 2 * (o + P)].view(2, P).cpu().numpy(),
            "normal": m0["normal"][3 * o: 3 * (o + P)].view(3, P).cpu().numpy(),
            "alpha": m0["alpha"][o: o + P].view(1, P).cpu().numpy(),
            "t_final": m0["t_final"][o: o + P].view(1, P).cpu().numpy(),
            "median": m0["median"][o: o + P].view(1, P).cpu().numpy(),
        }
        frag += compare_maps(g, ref, pixels=pix, check_int=False, label=f"view {vi} ")
        med = g["median"][0, pix]
        keep = (ref["fragile"] & 1) == 0
        assert np.array_equal(med[keep], ref["median_id"][keep])
    assert frag <= 2


def _loss_and_sig(st, views, scene, pix, gouts):
    rec, _, flags = oracle.project(st, views, scene)
    L, sig = 0.0, [flags.copy()]
    for vi, v in enumerate(views):
        out = oracle.render(st, v, rec[vi], flags[vi], pix[vi], want_sig=True)
        F = np.concatenate([out["color"], out["depth_exp"][:, None], out["depth_med"][:, None],
                            out["normal"], out["alpha"][:, None]], axis=1)
        L += float((F * gouts[vi]).sum())
        sig.append(out["sig"].copy())
    return L, sig


def test_recompute_gradients_on_2k_subsample_match_fp64_finite_differences():
    import torch
    from paper_2406_01467_amd.raster import Rasterizer
    dev = device()
    full, views = synth.make_workload(WORKLOAD)
    rng = np.random.default_rng(11)
    scene = full.subset(np.sort(rng.choice(full.n, 2000, replace=False)))
    del full
    s = _settings(sh_degree=3)
    st = oracle_settings(s)
    V = len(views)

    # Gaussians to differentiate: the largest footprints summed over views
    rec, rect, flags = oracle.project(st, views, scene)
    vis = (flags & oracle.F_VISIBLE) != 0
    area = np.where(vis, (rect[..., 1] - rect[..., 0] + 1) * (rect[..., 3] - rect[..., 2] + 1), 0)
    chosen = np.argsort(-area.sum(0))[:6]
    # pixels with upstream gradient: the chosen Gaussians' rects (capped)
    # plus a random sample, per view
    pix = []
    for vi, v in enumerate(views):
        sel = set(rng.choice(v.pixels, 256, replace=False).tolist())
        for g in chosen:
            if not vis[vi, g]:
                continue
            x0, x1, y0, y1 = rect[vi, g]
            ys, xs = np.mgrid[y0:y1 + 1, x0:x1 + 1]
            p = (ys * v.width + xs).reshape(-1)
            if p.size > 400:
                p = rng.choice(p, 400, replace=False)
            sel.update(p.tolist())
        pix.append(np.array(sorted(sel), np.int64))
    gouts = [rng.normal(size=(p.size, 9)) for p in pix]
    say("2k subsample:", V, "views,", sum(p.size for p in pix), "pixels with gradient; chosen",
        chosen.tolist(), "areas", area.sum(0)[chosen].tolist())

    # GPU: forward keeps no splats; backward recomputes them
    rast = Rasterizer(views, s, dev)
    params = to_dev(scene, dev)
    maps = rast.forward(*params, keep_splats=False)
    P = rast.total_pixels
    gC = np.zeros(3 * P, np.float32); gD = np.zeros(2 * P, np.float32)
    gN = np.zeros(3 * P, np.float32); gA = np.zeros(P, np.float32)
    for vi, v in enumerate(views):
        o, Pv, p, g = rast.views_c[vi].pix_offset, v.pixels, pix[vi], gouts[vi]
        for c in range(3):
            gC[3 * o + c * Pv + p] = g[:, c]
            gN[3 * o + c * Pv + p] = g[:, 5 + c]
        gD[2 * o + p] = g[:, 3]
        gD[2 * o + Pv + p] = g[:, 4]
        gA[o + p] = g[:, 8]
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    assert maps.state.splats is None
    dm, ds, dq, do, dsh = rast.backward(maps.state, *params, t(gC), t(gD), t(gN), t(gA))
    torch.cuda.synchronize()
    got = dict(means=dm.cpu().numpy(), scales=ds.cpu().numpy(), quats=dq.cpu().numpy(),
               opacities=do.cpu().numpy(), sh=dsh.cpu().numpy())

    # the FP64 adjoint, whole parameter set
    ref = oracle.backward(st, views, scene, gouts, pixels=pix)
    scale = oracle.gradient_error_scale(st, views, scene, gouts, pixels=pix)
    grad_check(got, ref, scale, "recompute 2k subsample")

    # FP64 central differences of the oracle forward, chosen Gaussians
    L0, sig0 = _loss_and_sig(st, views, scene, pix, gouts)
    entries = [("means", k) for k in range(3)] + [("scales", k) for k in range(3)] + \
        [("quats", k) for k in range(4)] + [("opacities", None)] + \
        [("sh", (0, c)) for c in range(3)] + [("sh", (6, 1))]
    checked = skipped = 0
    worst = 0.0
    for gi in chosen:
        for grp, k in entries:
            arr = getattr(scene, grp)
            idx = (gi,) if k is None else ((gi, k) if isinstance(k, int) else (gi,) + k)
            orig = float(arr[idx])
            h = 3e-5 * max(abs(orig), 1e-2)
            plus, minus = np.float32(orig + h), np.float32(orig - h)
            arr[idx] = plus
            Lp, sp = _loss_and_sig(st, views, scene, pix, gouts)
            arr[idx] = minus
            Lm, sm = _loss_and_sig(st, views, scene, pix, gouts)
            arr[idx] = np.float32(orig)
            if not (all(np.array_equal(a, b) for a, b in zip(sp, sig0)) and
                    all(np.array_equal(a, b) for a, b in zip(sm, sig0))):
                skipped += 1
                continue
            step = float(plus) - float(minus)
            fd = (Lp - Lm) / step
            g_gpu = float(np.asarray(got[grp]).reshape(arr.shape)[idx])
            S = float(np.asarray(scale[grp]).reshape(arr.shape)[idx])
            # GPU round-off bar (as above) + FD error: truncation ~1e-6
            # relative and FP64 round-off of L divided by the step
            bound = 1e-4 * (abs(fd) + 0.1 * S) + 1e-6 * abs(fd) + 1e-13 * (abs(L0) + 1) / step
            worst = max(worst, abs(g_gpu - fd) / bound)
            assert abs(g_gpu - fd) <= bound, (grp, int(gi), k, g_gpu, fd, S)
            checked += 1
    say(f"  finite differences: {checked} checked, {skipped} skipped by the discrete guard, "
        f"worst error / bound {worst:.3g}")
    assert checked >= 0.6 * (checked + skipped) and checked >= 40
