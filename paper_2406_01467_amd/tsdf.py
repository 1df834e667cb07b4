"""TSDF fusion of rendered median-depth maps (the mesh extraction of
Sec. 4.1) on top of the C ABI.  The grid is dense; at 8 bytes per voxel a
1024^3 grid takes 8.6 GB, which one MI355X holds many times over."""
from __future__ import annotations

import torch

from . import _lib


def tsdf_fuse(rast, depth: torch.Tensor, origin, voxel: float, dims, trunc: float):
    """Fuse the 2-plane depth maps `depth` that `rast` rendered into an
    nx x ny x nz grid (x fastest).  Returns (tsdf, weight), each (nz, ny, nx)."""
    nx, ny, nz = (int(d) for d in dims)
    tsdf = torch.empty(nz * ny * nx, dtype=torch.float32, device=depth.device)
    weight = torch.empty_like(tsdf)
    _lib.rade_tsdf_fuse(rast.settings, rast.views_c, rast.views_dev, depth.contiguous(), origin,
                        voxel, (nx, ny, nz), trunc, tsdf, weight)
    return tsdf.view(nz, ny, nx), weight.view(nz, ny, nx)
