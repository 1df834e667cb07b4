"""Pins of the oracle's Marching Cubes (Sec. 4.1, mesh extraction from the
fused TSDF) against geometry and topology: closed surfaces come out as
closed, consistently oriented manifolds with the Euler characteristic of
the shape, vertices lie on the level set (exactly for a linear field),
normals point up the field, and every cell configuration agrees with the
gradient of the trilinear interpolant."""
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle.mc import CORNERS, _edge_corners


def _grid(n, lo=-1.1, hi=1.1):
    h = (hi - lo) / n
    g = lo + (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    return X, Y, Z, np.full(3, lo), h


def _edges(tris):
    directed = Counter()
    for a, b, c in tris:
        for x, y in ((a, b), (b, c), (c, a)):
            directed[(int(x), int(y))] += 1
    undirected = Counter()
    for (x, y), m in directed.items():
        undirected[(min(x, y), max(x, y))] += m
    return directed, undirected


def _closed_oriented(tris):
    d, u = _edges(tris)
    assert max(d.values()) == 1, "a directed edge is used twice (orientation or manifold)"
    assert all(d[(y, x)] == 1 for (x, y) in d), "an edge with no opposite (a hole)"
    return u


def _mesh(f, n, o, h, w=None):
    w = np.ones(f.size) if w is None else w
    return oracle.marching_cubes(f.ravel(), w.ravel(), (n, n, n), o, h)


def test_sphere_closed_genus_zero_on_surface_outward():
    X, Y, Z, o, h = _grid(24)
    r0 = 0.8
    v, t, _ = _mesh(np.sqrt(X**2 + Y**2 + Z**2) - r0, 24, o, h)
    u = _closed_oriented(t)
    assert len(v) - len(u) + len(t) == 2
    r = np.linalg.norm(v, axis=1)
    # linear interpolation of a distance function along an edge of length h
    assert np.abs(r - r0).max() <= h * h / r0
    e1, e2 = v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]
    nrm = np.cross(e1, e2)
    assert np.all(np.sum(nrm * v[t].mean(1), 1) > 0)
    area = 0.5 * np.linalg.norm(nrm, axis=1).sum()
    assert abs(area / (4 * np.pi * r0**2) - 1) < 0.01


def test_torus_and_two_spheres_euler_characteristic():
    X, Y, Z, o, h = _grid(28)
    torus = np.sqrt((np.sqrt(X**2 + Y**2) - 0.6) ** 2 + Z**2) - 0.25
    v, t, _ = _mesh(torus, 28, o, h)
    u = _closed_oriented(t)
    assert len(v) - len(u) + len(t) == 0
    two = np.minimum(np.sqrt((X - 0.5) ** 2 + Y**2 + Z**2), np.sqrt((X + 0.5) ** 2 + Y**2 + Z**2)) - 0.3
    v, t, _ = _mesh(two, 28, o, h)
    u = _closed_oriented(t)
    assert len(v) - len(u) + len(t) == 4


def test_linear_field_gives_its_plane_exactly():
    X, Y, Z, o, h = _grid(13)
    nvec = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    f = nvec[0] * X + nvec[1] * Y + nvec[2] * Z - 0.1
    v, t, _ = _mesh(f, 13, o, h)
    assert len(t) > 100
    np.testing.assert_allclose(v @ nvec, 0.1, rtol=0, atol=1e-12)
    nrm = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    np.testing.assert_allclose(nrm @ nvec, 1.0, atol=1e-9)


def test_vertex_is_the_linear_zero_of_its_edge():
    rng = np.random.default_rng(3)
    n = 7
    f = rng.normal(size=(n, n, n))
    o, h = np.array([0.25, -1.0, 2.0]), 0.5
    v, t, e = oracle.marching_cubes(f.ravel(), np.ones(f.size), (n, n, n), o, h, iso=0.2)
    flat = f.ravel()
    step = {0: 1, 1: n, 2: n * n}
    for vi in range(0, len(e), 7):
        q, a = divmod(int(e[vi]), 3)
        i, j, k = q % n, (q // n) % n, q // (n * n)
        f0, f1 = flat[q], flat[q + step[a]]
        assert (f0 < 0.2) != (f1 < 0.2)
        s = (0.2 - f0) / (f1 - f0)
        want = o + (np.array([i, j, k]) + 0.5) * h
        want[a] += s * h
        np.testing.assert_allclose(v[vi], want, rtol=0, atol=1e-14)


def test_random_field_is_a_manifold_with_boundary_on_the_grid_faces():
    rng = np.random.default_rng(4)
    n = 12
    f = rng.normal(size=(n, n, n))
    v, t, e = oracle.marching_cubes(f.ravel(), np.ones(f.size), (n, n, n), np.zeros(3), 1.0)
    d, u = _edges(t)
    assert max(d.values()) == 1 and max(u.values()) <= 2
    # an edge used once lies on the grid's outer faces (both ends there)
    q, a = e // 3, e % 3
    idx = np.stack([q % n, (q // n) % n, q // (n * n)], 1)
    on_face = np.zeros(len(e), bool)
    for ax in range(3):
        other = idx[:, ax]
        on_face |= (other == 0) | (other == n - 1)
    shared_face = 0
    for (x, y), m in u.items():
        if m == 1:
            assert on_face[x] and on_face[y]
            shared_face += 1
    assert shared_face > 0


def test_unobserved_corners_mesh_nothing():
    X, Y, Z, o, h = _grid(16)
    f = np.sqrt(X**2 + Y**2 + Z**2) - 0.7
    assert len(_mesh(f, 16, o, h, np.zeros(f.shape))[1]) == 0
    w = np.ones(f.shape)
    w[X > 0.2] = 0.0
    v, t, e = _mesh(f, 16, o, h, w)
    full = _mesh(f, 16, o, h)
    assert 0 < len(t) < len(full[1])
    # every vertex lies on an edge whose ends were both observed
    q, a = e // 3, e % 3
    step = np.array([1, 16, 256])[a]
    assert np.all(w.ravel()[q] > 0) and np.all(w.ravel()[q + step] > 0)


@pytest.mark.parametrize("code", range(256))
def test_cell_configuration(code):
    """All 256 codes: the triangles use exactly the crossed edges, each of
    them at least once; normals follow the gradient of the trilinear
    interpolant of corner values -1 (inside) / +1 (outside) at the
    triangle's centroid; a code without a four-crossing face gives the
    reversed surface of its complement."""
    tris = oracle.cell_triangles(code)
    inside = [(code >> b) & 1 for b in range(8)]
    crossed = {e for e in range(12) if inside[_edge_corners(e)[0]] != inside[_edge_corners(e)[1]]}
    assert {e for tr in tris for e in tr} == crossed
    fv = np.array([-1.0 if s else 1.0 for s in inside])

    def grad(p):
        g = np.zeros(3)
        for b, c in enumerate(CORNERS):
            wts = [p[k] if c[k] else 1 - p[k] for k in range(3)]
            sgn = [1.0 if c[k] else -1.0 for k in range(3)]
            g += fv[b] * np.array([sgn[0] * wts[1] * wts[2], wts[0] * sgn[1] * wts[2],
                                   wts[0] * wts[1] * sgn[2]])
        return g

    def mid(e):
        c0, c1 = _edge_corners(e)
        return 0.5 * (np.array(CORNERS[c0], float) + np.array(CORNERS[c1], float))

    for tr in tris:
        p = [mid(e) for e in tr]
        nrm = np.cross(p[1] - p[0], p[2] - p[0])
        assert np.dot(nrm, grad(np.mean(p, 0))) > 0
    # faces: a diagonal pair of inside corners with the other two outside
    ambiguous = False
    for a in range(3):
        for side in (0, 1):
            ring = [c for c in range(8) if CORNERS[c][a] == side]
            vals = {tuple(CORNERS[c]): inside[c] for c in ring}
            ring_sorted = sorted(vals)
            s = [vals[p] for p in ring_sorted]
            ambiguous |= s[0] == s[3] and s[1] == s[2] and s[0] != s[1]
    if not ambiguous:
        comp = oracle.cell_triangles(255 - code)

        def canon(tr):
            k = tr.index(min(tr))
            return tr[k:] + tr[:k]
        assert {canon(tr) for tr in comp} == {canon(tr[::-1]) for tr in tris}
