"""Marching Cubes over a fused TSDF grid (the mesh extraction of Sec. 4.1:
a TSDF is built from the rendered depth maps and its zero level set is
extracted with Lorensen and Cline's Marching Cubes) -- TEST INFRASTRUCTURE
ONLY, FP64.

The per-cell triangulation is derived here from a rule, not from a printed
table:

* grid values sit at voxel centres; a cell is the cube between 2 x 2 x 2
  neighbouring centres, and is meshed only when all eight corners were
  observed (weight > 0);
* corner b of a cell sits at offset (b & 1, b >> 1 & 1, b >> 2 & 1); it is
  "inside" when its value is below the iso level; the cell code has bit b
  set for an inside corner;
* local edge (axis a, o1, o2) joins the two corners that differ along axis a
  and sit at offsets o1, o2 along the other two axes in increasing axis
  order; its index is 4 a + o1 + 2 o2;
* on each of the six faces, a face with two sign changes along its boundary
  carries one segment joining the two crossed edges; a face with four (the
  two inside corners diagonal) carries two segments, each cutting off one
  inside corner -- inside corners are never joined across a face, a choice
  that depends on the face alone and therefore agrees between the two cells
  sharing it (no cracks);
* each segment is directed so that, looking at the surface from the side
  where the field is above the iso level, the surface lies to its left
  (triangle normals then point up the field, out of the occupied region);
* every crossed edge starts exactly one segment and ends exactly one, so the
  segments form closed cycles, taken in the order of their smallest edge
  index; a cycle is cut into a fan from an apex whose chords (to the cycle's
  non-adjacent edges) all run through the cell's interior, i.e. join edges
  that share no face -- a chord lying in a face could be produced by the
  neighbouring cell too, and the mesh would not be a manifold there; the
  apex is the smallest such edge index (every cycle of the 256 codes has
  one), and the cycle (e0 = apex, e1, ..., ek-1) in segment direction gives
  the triangles (e0, ei, ei+1), i = 1 .. k-2.

Output: vertices are the crossed grid edges used by a meshed cell, in
increasing global edge id 3 q + a (q the voxel index, x fastest, a the axis
towards the next voxel), at the linear zero of the field along the edge;
triangles are taken cell by cell in increasing cell index (x fastest over
the nx - 1 cells of a row).
"""
from __future__ import annotations

import functools

import numpy as np

CORNERS = [(b & 1, (b >> 1) & 1, (b >> 2) & 1) for b in range(8)]


def _others(a):
    return [x for x in range(3) if x != a]


def _edge_corners(e):
    """The two corner ids joined by local edge e (lower end first)."""
    a, o1, o2 = e // 4, e % 2, (e // 2) % 2
    u, v = _others(a)
    lo = [0, 0, 0]
    lo[u], lo[v] = o1, o2
    hi = list(lo)
    hi[a] = 1
    cid = lambda p: p[0] + 2 * p[1] + 4 * p[2]  # noqa: E731
    return cid(lo), cid(hi)


def _edge_between(c0, c1):
    p, q = CORNERS[c0], CORNERS[c1]
    a = [k for k in range(3) if p[k] != q[k]]
    assert len(a) == 1
    a = a[0]
    u, v = _others(a)
    return 4 * a + p[u] + 2 * p[v]


def _faces():
    """(outward normal, four corner ids in cyclic order) per face."""
    out = []
    for a in range(3):
        u, v = _others(a)
        for side in (0, 1):
            ring = []
            for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):
                p = [0, 0, 0]
                p[a], p[u], p[v] = side, du, dv
                ring.append(p[0] + 2 * p[1] + 4 * p[2])
            n = np.zeros(3)
            n[a] = 1.0 if side else -1.0
            out.append((n, ring))
    return out


def _edge_faces(e):
    c0, c1 = _edge_corners(e)
    return {fi for fi, (_, ring) in enumerate(_faces()) if c0 in ring and c1 in ring}


def _share_face(a, b):
    return bool(_edge_faces(a) & _edge_faces(b))


def _mid(e):
    c0, c1 = _edge_corners(e)
    return 0.5 * (np.array(CORNERS[c0], float) + np.array(CORNERS[c1], float))


@functools.lru_cache(maxsize=None)
def cell_triangles(code: int):
    """Triangles (triples of local edge ids) of a cell with this code."""
    inside = [(code >> b) & 1 for b in range(8)]
    nxt = {}
    for n, ring in _faces():
        pos = [np.array(CORNERS[c], float) for c in ring]
        edges = [_edge_between(ring[k], ring[(k + 1) % 4]) for k in range(4)]
        cross = [inside[ring[k]] != inside[ring[(k + 1) % 4]] for k in range(4)]
        segs = []  # (edge A, edge B, direction from the inside side to the outside side)
        if sum(cross) == 2:
            A, B = [edges[k] for k in range(4) if cross[k]]
            pin = np.mean([pos[k] for k in range(4) if inside[ring[k]]], axis=0)
            pout = np.mean([pos[k] for k in range(4) if not inside[ring[k]]], axis=0)
            segs.append((A, B, pout - pin))
        elif sum(cross) == 4:
            centre = np.mean(pos, axis=0)
            for k in range(4):
                if inside[ring[k]]:
                    segs.append((edges[k - 1], edges[k], centre - pos[k]))
        for A, B, g in segs:
            # the surface's up-field normal has the in-face component g; the
            # boundary runs along g x n (surface on its left seen from there)
            if np.dot(_mid(B) - _mid(A), np.cross(g, n)) < 0:
                A, B = B, A
            assert A not in nxt
            nxt[A] = B
    assert sorted(nxt) == sorted(nxt.values())
    tris = []
    seen = set()
    for start in sorted(nxt):
        if start in seen:
            continue
        cyc = [start]
        seen.add(start)
        e = nxt[start]
        while e != start:
            cyc.append(e)
            seen.add(e)
            e = nxt[e]
        k = len(cyc)
        clean = [cyc[a] for a in range(k)
                 if not any(_share_face(cyc[a], cyc[b]) for b in range(k)
                            if b not in (a, (a + 1) % k, (a - 1) % k))]
        r = cyc.index(min(clean))
        cyc = cyc[r:] + cyc[:r]
        for i in range(1, k - 1):
            tris.append((cyc[0], cyc[i], cyc[i + 1]))
    return tuple(tris)


def _local_to_global(e, i, j, k, nx, ny):
    a, o1, o2 = e // 4, e % 2, (e // 2) % 2
    p = [i, j, k]
    u, v = _others(a)
    p[u] += o1
    p[v] += o2
    return 3 * ((p[2] * ny + p[1]) * nx + p[0]) + a


def marching_cubes(tsdf, weight, dims, origin, voxel, iso=0.0):
    """Mesh of the iso level of a grid (values and weights of nx * ny * nz
    voxels, x fastest, centres at origin + (i + 1/2) voxel).  Returns
    (vertices (nv, 3) FP64, triangles (nt, 3) int64, global edge id of each
    vertex)."""
    nx, ny, nz = (int(d) for d in dims)
    f = np.asarray(tsdf, np.float64).reshape(nz, ny, nx)
    w = np.asarray(weight, np.float64).reshape(nz, ny, nx)
    o = np.asarray(origin, np.float64)
    tris_edges = []
    if nx >= 2 and ny >= 2 and nz >= 2:
        sl = lambda d: slice(d, None) if d else slice(None, -1)  # noqa: E731
        valid = np.ones((nz - 1, ny - 1, nx - 1), bool)
        code = np.zeros((nz - 1, ny - 1, nx - 1), np.int64)
        for b, (dx, dy, dz) in enumerate(CORNERS):
            valid &= w[sl(dz), sl(dy), sl(dx)] > 0
            code |= (f[sl(dz), sl(dy), sl(dx)] < iso).astype(np.int64) << b
        for k, j, i in zip(*np.nonzero(valid & (code != 0) & (code != 255))):
            for t in cell_triangles(int(code[k, j, i])):
                tris_edges.append([_local_to_global(e, i, j, k, nx, ny) for e in t])
    tris_edges = np.array(tris_edges, np.int64).reshape(-1, 3)
    # rows of the triangle list follow the cell index, as nonzero() returns
    # cells in (k, j, i) order, i.e. increasing x-fastest index
    edges = np.unique(tris_edges)
    tris = np.searchsorted(edges, tris_edges).astype(np.int64)
    q, a = edges // 3, edges % 3
    idx = np.stack([q % nx, (q // nx) % ny, q // (nx * ny)], axis=1)
    step = np.array([1, nx, nx * ny])[a]
    f0 = f.reshape(-1)[q]
    f1 = f.reshape(-1)[q + step]
    t = (iso - f0) / (f1 - f0)
    verts = o + (idx + 0.5) * voxel
    verts[np.arange(len(edges)), a] += t * voxel
    return verts, tris, edges
