"""Marching Cubes over a TSDF grid (the mesh extraction of Sec. 4.1) on top
of the C ABI: the triangle mesh of the grid's iso level, vertices in FP32,
triangles as int32 vertex indices (normals up the field)."""
from __future__ import annotations

import torch

from . import _lib


def marching_cubes(tsdf: torch.Tensor, weight: torch.Tensor, origin, voxel: float,
                   iso: float = 0.0, capacity=None, stream=None):
    """tsdf, weight: (nz, ny, nx) float32 device tensors (x fastest), as
    `tsdf.tsdf_fuse` returns them.  Returns (verts (nv, 3) float32, tris (nt,
    3) int32).  Output buffers start at `capacity` = (verts, tris) or a guess
    from the grid's face areas and grow once to the exact size when the
    surface is larger (the library reports the counts)."""
    nz, ny, nx = (int(d) for d in tsdf.shape)
    dims = (nx, ny, nz)
    dev = tsdf.device
    ws = torch.empty(max(_lib.rade_marching_cubes_workspace(dims), 1), dtype=torch.uint8,
                     device=dev)
    if capacity is None:
        cv = min(3 * nx * ny * nz, 4 * (nx * ny + ny * nz + nz * nx))
        capacity = (cv, 2 * cv)
    cv, ct = (int(c) for c in capacity)
    f = tsdf.contiguous()
    w = weight.contiguous()
    for _ in range(2):
        verts = torch.empty(max(cv, 1) * 3, dtype=torch.float32, device=dev)
        tris = torch.empty(max(ct, 1) * 3, dtype=torch.int32, device=dev)
        code, nv, nt = _lib.rade_marching_cubes(f, w, dims, origin, voxel, iso, ws, verts, cv,
                                                tris, ct, stream)
        if code == _lib.RADE_OK:
            return verts[:3 * nv].view(nv, 3), tris[:3 * nt].view(nt, 3)
        cv, ct = nv, nt
    raise RuntimeError("rade_marching_cubes: capacity still exceeded after resizing")
