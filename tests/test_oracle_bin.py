"""Pins of the binning reference by brute force on small inputs: every (tile,
Gaussian) pair whose pixel rect touches the tile, each tile's list in
ascending (float32 depth, id) order."""
import numpy as np
import pytest

import oracle
import synth


def _brute(views, rect, z, tile):
    lists = []
    for vi, v in enumerate(views):
        tx_n = (v.width + tile[0] - 1) // tile[0]
        ty_n = (v.height + tile[1] - 1) // tile[1]
        for ty in range(ty_n):
            for tx in range(tx_n):
                x0, x1 = tx * tile[0], tx * tile[0] + tile[0] - 1
                y0, y1 = ty * tile[1], ty * tile[1] + tile[1] - 1
                ids = [g for g in range(rect.shape[1])
                       if rect[vi, g, 0] <= rect[vi, g, 1] and rect[vi, g, 2] <= rect[vi, g, 3]
                       and rect[vi, g, 0] <= x1 and rect[vi, g, 1] >= x0
                       and rect[vi, g, 2] <= y1 and rect[vi, g, 3] >= y0]
                ids.sort(key=lambda g: (float(z[vi, g]), g))
                lists.append(ids)
    return lists


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (16, 32), (32, 16)])
def test_bin_matches_brute_force(tile):
    rng = np.random.default_rng(tile[0] * 7 + tile[1])
    views = [synth.identity_view(70, 45), synth.identity_view(33, 64)]
    N = 120
    rect = np.zeros((2, N, 4), np.int32)
    for vi, v in enumerate(views):
        x0 = rng.integers(0, v.width, N)
        y0 = rng.integers(0, v.height, N)
        rect[vi, :, 0] = x0
        rect[vi, :, 1] = np.minimum(v.width - 1, x0 + rng.integers(0, 30, N))
        rect[vi, :, 2] = y0
        rect[vi, :, 3] = np.minimum(v.height - 1, y0 + rng.integers(0, 30, N))
    rect[:, ::7, 1] = -1  # some invisible
    # depths with deliberate ties
    z = rng.choice(np.array([1.5, 2.0, 2.25, 3.0], np.float32), size=(2, N))
    ids, keys, ranges = oracle.bin_pairs(views, rect, z, tile)
    lists = _brute(views, rect, z, tile)
    assert ranges.shape[0] == len(lists)
    for t, want in enumerate(lists):
        s, e = ranges[t]
        got = list(ids[s:e]) if e > s else []
        assert got == want, t
        for i in range(s, e):
            assert int(keys[i]) >> 32 == t
    assert len(ids) == sum(len(x) for x in lists)
    # keys are sorted and carry the float bits of z in the low word
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)


def test_bin_of_projected_scene_covers_contributors():
    # Every Gaussian that contributes to a pixel is in that pixel's tile list.
    scene, views = synth.make_workload("plain_64x64_1k")
    st = oracle.settings()
    rec, rect, flags = oracle.project(st, views, scene)
    z = rec[:, :, oracle.R["z"]].astype(np.float32)
    ids, keys, ranges = oracle.bin_pairs(views, rect, z, (16, 16))
    v = views[0]
    tiles_x = (v.width + 15) // 16
    # single-Gaussian renders: alpha > 0 only inside the tiles that list it
    in_tiles = {}
    for t in range(ranges.shape[0]):
        for g in ids[ranges[t, 0]:ranges[t, 1]]:
            in_tiles.setdefault(int(g), set()).add(t)
    for g in range(0, scene.n, 37):
        if flags[0, g] & oracle.F_CULLED:
            continue
        out = oracle.render(st, v, rec[0][g:g + 1], flags[0][g:g + 1])
        hit = np.flatnonzero(out["count"] > 0)
        tiles = {(p // v.width) // 16 * tiles_x + (p % v.width) // 16 for p in hit}
        assert tiles <= in_tiles.get(g, set())
