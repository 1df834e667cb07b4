"""The allocation-free normal-consistency entry point against the one that
takes a workspace: same kernels, so the loss and the three gradient maps must
agree bit for bit, on two calls in a row (the second on a smaller input, so
it reads partials the first call left behind only if it indexes wrongly),
in both the accumulate and the overwrite mode."""
import numpy as np
import pytest

from gpu_common import device, say

pytestmark = pytest.mark.gpu


def _maps(views, seed):
    """Seeded maps of the prepared views: a smooth median depth with noise,
    random normals and alphas (only their shapes matter here)."""
    rng = np.random.default_rng(seed)
    depth, normal, alpha = [], [], []
    for w, h in views:
        yy, xx = np.mgrid[0:h, 0:w]
        d = 3.0 + 0.3 * np.sin(xx / 17.0) + 0.2 * np.cos(yy / 11.0) + 0.01 * rng.normal(size=(h, w))
        depth += [rng.uniform(1, 5, h * w), d.reshape(-1)]
        normal += [rng.normal(size=3 * h * w)]
        alpha += [rng.uniform(0, 1, h * w)]
    # planar layout per view: depth 2 planes, normal 3, alpha 1, views back to back
    return (np.concatenate(depth).astype(np.float32), np.concatenate(normal).astype(np.float32),
            np.concatenate(alpha).astype(np.float32))


def _both(sizes, seed, accumulate, dev):
    import torch
    import synth
    from paper_2406_01467_amd import _lib
    views = [synth.identity_view(w, h) for w, h in sizes]
    vc = _lib.make_views(views)
    P, _ = _lib.rade_views_prepare(_lib.Settings(), vc)
    vdev = _lib.views_to_device(vc, dev)
    depth, normal, alpha = _maps(sizes, seed)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    D, N, A = t(depth), t(normal), t(alpha)
    rng = np.random.default_rng(seed + 1)
    base = [rng.normal(size=k * P).astype(np.float32) for k in (2, 3, 1)]
    out = []
    for noalloc in (False, True):
        loss = torch.full((len(sizes),), float("nan"), device=dev)
        grads = [t(b) for b in base]
        if noalloc:
            _lib.rade_normal_consistency_noalloc(vc, vdev, D, N, A, 5.0, loss, *grads,
                                                 accumulate=accumulate)
        else:
            ws = torch.empty(_lib.rade_normal_consistency_workspace(P), dtype=torch.uint8,
                             device=dev)
            _lib.rade_normal_consistency(vc, vdev, D, N, A, 5.0, loss, *grads, ws,
                                         accumulate=accumulate)
        torch.cuda.synchronize()
        out.append([loss.cpu().numpy()] + [g.cpu().numpy() for g in grads])
    return out


@pytest.mark.parametrize("accumulate", [True, False])
def test_noalloc_normal_consistency_matches_the_workspace_form(accumulate):
    dev = device()
    for k, (sizes, seed) in enumerate((([(300, 200), (128, 77), (61, 45)], 5), ([(50, 40)], 6))):
        say(f"call {k}: views {sizes}, accumulate {accumulate}")
        ref, got = _both(sizes, seed, accumulate, dev)
        assert np.all(np.isfinite(ref[0]))
        for name, r, g in zip(("loss", "d_depth", "d_normal", "d_alpha"), ref, got):
            assert np.array_equal(r.view(np.uint32), g.view(np.uint32)), (k, name)


def test_noalloc_rejects_more_blocks_than_its_scratch():
    import torch
    import synth
    from paper_2406_01467_amd import _lib
    dev = device()
    vc = _lib.make_views([synth.identity_view(8192, 8192)])  # 256 x 1024 blocks
    _lib.rade_views_prepare(_lib.Settings(), vc)
    vdev = _lib.views_to_device(vc, dev)
    x = torch.zeros(8, device=dev)
    with pytest.raises(_lib.RadeError) as e:
        _lib.rade_normal_consistency_noalloc(vc, vdev, x, x, x, 1.0, x, x, x, x)
    assert e.value.code == _lib.RADE_ERR_TOO_LARGE
