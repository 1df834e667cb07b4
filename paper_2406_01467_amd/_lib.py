"""ctypes binding of librade.so (include/rade.h).

Argument marshalling only: every step of the rasterizer runs in the HIP
kernels of librade.so.  Functions keep the C names and take torch tensors
(device memory) plus host-side view/setting objects.  Loading fails loudly
when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# RADE_LIBRARY selects another build of the library (e.g. a debug build).
LIB_PATH = os.environ.get("RADE_LIBRARY") or os.path.join(HERE, "librade.so")

RADE_OK = 0
RADE_ERR_INVALID_ARG = -1
RADE_ERR_CAPACITY = -2
RADE_ERR_HIP = -3
RADE_ERR_UNSUPPORTED_DEVICE = -4
RADE_ERR_WORKSPACE = -5
RADE_ERR_TOO_LARGE = -6
RADE_NC_NOALLOC_MAX_BLOCKS = 131072

RADE_SCHEDULE_TILE, RADE_SCHEDULE_HEAVY_FIRST, RADE_SCHEDULE_PERSISTENT = 0, 1, 2

SPLAT_BYTES = 80
GRAD_FLOATS = 16

# NumPy view of struct rade_splat (80 bytes).
SPLAT_DTYPE = np.dtype([("uc", "<f8"), ("vc", "<f8"), ("w", "<f4", (4,)), ("opacity", "<f4"),
                        ("rgb", "<f4", (3,)), ("z", "<f4"), ("p", "<f4", (2,)),
                        ("n", "<f4", (3,)), ("rect", "<i2", (4,))])
assert SPLAT_DTYPE.itemsize == SPLAT_BYTES


class RadeError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class CSettings(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("dilation", ctypes.c_double), ("near_plane", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("t_min", ctypes.c_double), ("power_cut", ctypes.c_double),
                ("fov_clamp", ctypes.c_double), ("degenerate", ctypes.c_double),
                ("bg", ctypes.c_double * 3), ("depth_mode", ctypes.c_int32),
                ("wave_w", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lane_masks", ctypes.c_int32)]


class CView(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("pix_offset", ctypes.c_int64), ("tile_offset", ctypes.c_int64)]


assert ctypes.sizeof(CView) == 96 and ctypes.sizeof(CSettings) == 120

RADE_DEPTH_AFFINE, RADE_DEPTH_EXACT = 0, 1


@dataclasses.dataclass
class Settings:
    """Mirror of rade_settings; defaults are the 3DGS defaults the paper keeps."""
    tile_w: int = 16
    tile_h: int = 16
    sh_degree: int = 0
    schedule: int = 0          # RADE_SCHEDULE_*
    dilation: float = 0.3
    near_plane: float = 0.2
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    power_cut: float = 4.5
    fov_clamp: float = 1.3
    degenerate: float = 1e-6
    bg: tuple = (0.0, 0.0, 0.0)
    depth_mode: int = 0        # RADE_DEPTH_AFFINE (Eq. 4) or RADE_DEPTH_EXACT (Eq. 7, forward only)
    wave_w: int = 0            # pixels per wave row: 8 (8x8), 16 (16x4), 32 (32x2); 0 = 8
    batch: int = 0             # splats staged per round: 64..512; 0 = tile_w * tile_h
    lane_masks: int = 0        # 1: per-wave lane masks on tiles of several 8x8 waves

    def c(self) -> CSettings:
        s = CSettings()
        s.tile_w, s.tile_h, s.sh_degree = self.tile_w, self.tile_h, self.sh_degree
        s.schedule = self.schedule
        s.dilation, s.near_plane = self.dilation, self.near_plane
        s.alpha_min, s.alpha_max, s.t_min = self.alpha_min, self.alpha_max, self.t_min
        s.power_cut, s.fov_clamp, s.degenerate = self.power_cut, self.fov_clamp, self.degenerate
        for i in range(3):
            s.bg[i] = float(self.bg[i])
        s.depth_mode, s.wave_w, s.batch = self.depth_mode, self.wave_w, self.batch
        s.lane_masks = self.lane_masks
        return s


_lib = None
ABI_VERSION = 8


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2406_01467_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.rade_views_prepare.argtypes = [P, P, I32, P, P]
    lib.rade_project.argtypes = [P, P, I32, I64] + [P] * 9 + [P]
    lib.rade_bin_sort_workspace.argtypes = [I32, I64, I64, I64]
    lib.rade_bin_sort_workspace.restype = SZ
    lib.rade_bin_sort.argtypes = [P, P, P, I32, I64, P, P, P, P, P, I64, P, P, P, SZ, P]
    lib.rade_render_fwd.argtypes = [P, P, P, I32, I64] + [P] * 16 + [P]
    lib.rade_lane_mask_bytes.argtypes = [P, I64]
    lib.rade_lane_mask_bytes.restype = SZ
    lib.rade_tile_order_workspace.argtypes = [I64]
    lib.rade_tile_order_workspace.restype = SZ
    lib.rade_tile_order.argtypes = [P, P, I32, P, P, P, SZ, P]
    lib.rade_tile_order.restype = ctypes.c_int
    lib.rade_render_bwd_workspace.argtypes = [P, I32, I64, ctypes.c_int]
    lib.rade_render_bwd_workspace.restype = SZ
    lib.rade_render_bwd.argtypes = [P, P, P, I32, I64] + [P] * 26 + [SZ, P]
    lib.rade_strerror.argtypes = [ctypes.c_int]
    lib.rade_strerror.restype = ctypes.c_char_p
    lib.rade_abi_version.restype = ctypes.c_int
    lib.rade_device_check.argtypes = []
    lib.rade_device_check.restype = ctypes.c_int
    if lib.rade_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} implements ABI {lib.rade_abi_version()}, this binding "
                           f"needs {ABI_VERSION}: rebuild with `python -m paper_2406_01467_amd.build`")
    lib.rade_set_kernel_events.argtypes = [ctypes.c_int, P, P]
    lib.rade_normal_consistency_workspace.argtypes = [I64]
    lib.rade_normal_consistency_workspace.restype = SZ
    lib.rade_normal_consistency.argtypes = [P, P, I32] + [P] * 3 + [ctypes.c_float] + [P] * 4 + \
        [I32, P, SZ, P]
    lib.rade_normal_consistency_noalloc.argtypes = [P, P, I32] + [P] * 3 + [ctypes.c_float] + \
        [P] * 4 + [I32, P]
    lib.rade_normal_consistency_noalloc.restype = ctypes.c_int
    lib.rade_l1_color_grad.argtypes = [P, P, I32, P, P, ctypes.c_float, P, P]
    lib.rade_l1_color_grad.restype = ctypes.c_int
    lib.rade_normal_consistency.restype = ctypes.c_int
    lib.rade_set_kernel_events.restype = ctypes.c_int
    lib.rade_filter3d_var.argtypes = [P, P, I32, I64, P, ctypes.c_float, ctypes.c_float, P, P]
    lib.rade_filter3d_apply.argtypes = [I64] + [P] * 5 + [P]
    lib.rade_filter3d_apply_bwd.argtypes = [I64] + [P] * 7 + [P]
    lib.rade_tsdf_fuse.argtypes = [P, P, P, I32, P, P, ctypes.c_double, I32, I32, I32,
                                   ctypes.c_float, P, P, P]
    lib.rade_marching_cubes_workspace.argtypes = [I32, I32, I32]
    lib.rade_marching_cubes_workspace.restype = SZ
    lib.rade_marching_cubes.argtypes = [P, P, I32, I32, I32, P, ctypes.c_double, ctypes.c_float,
                                        P, SZ, P, I64, P, I64, P, P, P]
    lib.rade_marching_cubes_table.argtypes = [P, P]
    for f in ("rade_filter3d_var", "rade_filter3d_apply", "rade_filter3d_apply_bwd",
              "rade_tsdf_fuse", "rade_marching_cubes", "rade_marching_cubes_table"):
        getattr(lib, f).restype = ctypes.c_int
    for f in ("rade_views_prepare", "rade_project", "rade_bin_sort", "rade_render_fwd",
              "rade_render_bwd"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


EXPORTED = ["rade_views_prepare", "rade_project", "rade_bin_sort_workspace", "rade_bin_sort",
            "rade_render_fwd", "rade_lane_mask_bytes", "rade_render_bwd_workspace", "rade_render_bwd", "rade_strerror",
            "rade_abi_version", "rade_set_kernel_events", "rade_tile_order_workspace",
            "rade_tile_order", "rade_normal_consistency_workspace", "rade_normal_consistency",
            "rade_filter3d_var", "rade_filter3d_apply", "rade_filter3d_apply_bwd",
            "rade_tsdf_fuse", "rade_marching_cubes_workspace", "rade_marching_cubes",
            "rade_marching_cubes_table", "rade_l1_color_grad", "rade_device_check",
            "rade_normal_consistency_noalloc"]

RADE_KERNEL_PROJECT, RADE_KERNEL_RENDER_FWD, RADE_KERNEL_RENDER_BWD, RADE_KERNEL_PROJECT_BWD = 1, 2, 3, 4


def rade_set_kernel_events(kernel: int, start=None, stop=None):
    """start/stop: torch.cuda.Event (created with enable_timing=True) or None."""
    sp = None if start is None else ctypes.c_void_p(start.cuda_event)
    ep = None if stop is None else ctypes.c_void_p(stop.cuda_event)
    return _check(load().rade_set_kernel_events(kernel, sp, ep), "rade_set_kernel_events")


def strerror(code: int) -> str:
    try:
        return load().rade_strerror(code).decode()
    except Exception:  # noqa: BLE001 - message only
        return "error"


def _check(code: int, what: str) -> int:
    if code != RADE_OK:
        raise RadeError(code, what)
    return code


def _p(t):
    """Device (or host) address of a tensor / ndarray, or None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return ctypes.c_void_p(t.ctypes.data)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def make_views(views: Sequence) -> ctypes.Array:
    """Host array of rade_view from objects with width, height, fx, fy, cx,
    cy, R (3x3), t (3)."""
    arr = (CView * len(views))()
    for i, v in enumerate(views):
        c = arr[i]
        c.width, c.height = int(v.width), int(v.height)
        c.fx, c.fy, c.cx, c.cy = float(v.fx), float(v.fy), float(v.cx), float(v.cy)
        R = np.asarray(v.R, np.float32).reshape(9)
        t = np.asarray(v.t, np.float32).reshape(3)
        for k in range(9):
            c.R[k] = float(R[k])
        for k in range(3):
            c.t[k] = float(t[k])
    return arr


def rade_views_prepare(settings: Settings, views_c: ctypes.Array):
    s = settings.c()
    tp, tt = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load().rade_views_prepare(ctypes.byref(s), views_c, len(views_c), ctypes.byref(tp),
                                     ctypes.byref(tt)), "rade_views_prepare")
    return tp.value, tt.value


def views_to_device(views_c: ctypes.Array, device):
    import torch
    raw = np.frombuffer(bytes(views_c), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


def rade_project(settings: Settings, views_dev, V: int, N: int, means, scales, quats, opacities,
                 sh, splats, tiles_touched, stream=None, depth_quad=None, bin_records=None):
    s = settings.c()
    return _check(load().rade_project(ctypes.byref(s), _p(views_dev), V, N, _p(means), _p(scales),
                                      _p(quats), _p(opacities), _p(sh), _p(splats),
                                      _p(tiles_touched), _p(bin_records), _p(depth_quad),
                                      _stream(stream)),
                  "rade_project")


def rade_bin_sort_workspace(V: int, N: int, capacity: int, total_tiles: int) -> int:
    return int(load().rade_bin_sort_workspace(V, N, capacity, total_tiles))


def rade_bin_sort(settings: Settings, views_c, views_dev, V: int, N: int, tiles_touched,
                  bin_records, pair_ids, tile_ranges, keys, capacity: int, n_pairs_dev, workspace,
                  stream=None, sync_count: bool = True):
    """Returns (status, M) where M is the pair count when sync_count, else None.
    Raises on any error except RADE_ERR_CAPACITY (returned as status)."""
    s = settings.c()
    host = ctypes.c_int64(-1)
    code = load().rade_bin_sort(ctypes.byref(s), views_c, _p(views_dev), V, N,
                                _p(tiles_touched), _p(bin_records), _p(pair_ids),
                                _p(tile_ranges), _p(keys),
                                capacity, _p(n_pairs_dev),
                                ctypes.byref(host) if sync_count else None, _p(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream))
    if code not in (RADE_OK, RADE_ERR_CAPACITY):
        _check(code, "rade_bin_sort")
    return code, (host.value if sync_count else None)


def rade_tile_order_workspace(total_tiles: int) -> int:
    return int(load().rade_tile_order_workspace(total_tiles))


def rade_tile_order(settings: Settings, views_c, tile_ranges, tile_order, workspace, stream=None):
    s = settings.c()
    return _check(load().rade_tile_order(ctypes.byref(s), views_c, len(views_c), _p(tile_ranges),
                                         _p(tile_order), _p(workspace),
                                         workspace.numel() * workspace.element_size(),
                                         _stream(stream)), "rade_tile_order")


def rade_render_fwd(settings: Settings, views_c, views_dev, V: int, N: int, splats, pair_ids,
                    tile_ranges, color, depth, normal, alpha, t_final, last, median, count=None,
                    stream=None, tile_order=None, distortion=None, depth_quad=None, evals=None,
                    lane_masks=None):
    """lane_masks (optional): the cache of rade_lane_mask_bytes(settings, pairs)
    bytes the forward fills for the backward."""
    s = settings.c()
    return _check(load().rade_render_fwd(ctypes.byref(s), views_c, _p(views_dev), V, N,
                                         _p(splats), _p(pair_ids), _p(tile_ranges),
                                         _p(tile_order), _p(color),
                                         _p(depth), _p(normal), _p(alpha), _p(t_final), _p(last),
                                         _p(median), _p(count), _p(evals), _p(distortion),
                                         _p(depth_quad), _p(lane_masks), _stream(stream)),
                  "rade_render_fwd")


def rade_device_check() -> int:
    """RADE_OK when the current HIP device is a gfx950 GPU, else
    RADE_ERR_UNSUPPORTED_DEVICE (returned, not raised)."""
    return int(load().rade_device_check())


def rade_lane_mask_bytes(settings: Settings, n_pairs: int) -> int:
    """Bytes of the forward's lane-mask cache for n_pairs list entries (0 where
    the launch shape keeps no lane masks)."""
    s = settings.c()
    return int(load().rade_lane_mask_bytes(ctypes.byref(s), int(n_pairs)))


def rade_render_bwd_workspace(settings: Settings, V: int, N: int, recompute: bool) -> int:
    s = settings.c()
    return int(load().rade_render_bwd_workspace(ctypes.byref(s), V, N, 1 if recompute else 0))


def rade_render_bwd(settings: Settings, views_c, views_dev, V: int, N: int, means, scales, quats,
                    opacities, sh, splats, pair_ids, tile_ranges, t_final, last, median, d_color,
                    d_depth, d_normal, d_alpha, d_means, d_scales, d_quats, d_opacities, d_sh,
                    workspace, stream=None, tile_order=None, d_distortion=None, depth=None,
                    alpha=None, lane_masks=None):
    """d_distortion (optional) needs the forward's depth (2 planes) and alpha maps;
    lane_masks (optional): the cache the forward filled for the same lists."""
    s = settings.c()
    return _check(load().rade_render_bwd(
        ctypes.byref(s), views_c, _p(views_dev), V, N, _p(means), _p(scales), _p(quats),
        _p(opacities), _p(sh), _p(splats), _p(pair_ids), _p(tile_ranges), _p(tile_order),
        _p(t_final), _p(last),
        _p(median), _p(d_color), _p(d_depth), _p(d_normal), _p(d_alpha), _p(d_distortion),
        _p(depth), _p(alpha), _p(lane_masks), _p(d_means),
        _p(d_scales), _p(d_quats), _p(d_opacities), _p(d_sh), _p(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)), "rade_render_bwd")


def rade_normal_consistency_workspace(total_pixels: int) -> int:
    return int(load().rade_normal_consistency_workspace(total_pixels))


def rade_normal_consistency(views_c, views_dev, depth, normal, alpha, weight: float, loss, d_depth,
                            d_normal, d_alpha, workspace, stream=None, accumulate: bool = True):
    return _check(load().rade_normal_consistency(
        views_c, _p(views_dev), len(views_c), _p(depth), _p(normal), _p(alpha), float(weight),
        _p(loss), _p(d_depth), _p(d_normal), _p(d_alpha), 1 if accumulate else 0, _p(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)), "rade_normal_consistency")


def rade_normal_consistency_noalloc(views_c, views_dev, depth, normal, alpha, weight: float, loss,
                                    d_depth, d_normal, d_alpha, stream=None,
                                    accumulate: bool = True):
    return _check(load().rade_normal_consistency_noalloc(
        views_c, _p(views_dev), len(views_c), _p(depth), _p(normal), _p(alpha), float(weight),
        _p(loss), _p(d_depth), _p(d_normal), _p(d_alpha), 1 if accumulate else 0,
        _stream(stream)), "rade_normal_consistency_noalloc")


def rade_l1_color_grad(views_c, views_dev, color, target, weight: float, d_color, stream=None):
    return _check(load().rade_l1_color_grad(views_c, _p(views_dev), len(views_c), _p(color),
                                            _p(target), float(weight), _p(d_color),
                                            _stream(stream)), "rade_l1_color_grad")


def rade_filter3d_var(settings: Settings, views_dev, V: int, N: int, means, scale: float,
                      margin: float, var, stream=None):
    s = settings.c()
    return _check(load().rade_filter3d_var(ctypes.byref(s), _p(views_dev), V, N, _p(means),
                                           float(scale), float(margin), _p(var),
                                           _stream(stream)), "rade_filter3d_var")


def rade_filter3d_apply(N: int, scales, opacities, var, scales_out, opacities_out, stream=None):
    return _check(load().rade_filter3d_apply(N, _p(scales), _p(opacities), _p(var),
                                             _p(scales_out), _p(opacities_out), _stream(stream)),
                  "rade_filter3d_apply")


def rade_filter3d_apply_bwd(N: int, scales, opacities, var, d_scales_out, d_opacities_out,
                            d_scales, d_opacities, stream=None):
    return _check(load().rade_filter3d_apply_bwd(N, _p(scales), _p(opacities), _p(var),
                                                 _p(d_scales_out), _p(d_opacities_out),
                                                 _p(d_scales), _p(d_opacities), _stream(stream)),
                  "rade_filter3d_apply_bwd")


def rade_tsdf_fuse(settings: Settings, views_c, views_dev, depth, origin, voxel: float, dims,
                   trunc: float, tsdf, weight, stream=None):
    s = settings.c()
    o = (ctypes.c_double * 3)(*[float(x) for x in origin])
    nx, ny, nz = (int(d) for d in dims)
    return _check(load().rade_tsdf_fuse(ctypes.byref(s), views_c, _p(views_dev), len(views_c),
                                        _p(depth), o, float(voxel), nx, ny, nz, float(trunc),
                                        _p(tsdf), _p(weight), _stream(stream)), "rade_tsdf_fuse")


def rade_marching_cubes_workspace(dims) -> int:
    nx, ny, nz = (int(d) for d in dims)
    return int(load().rade_marching_cubes_workspace(nx, ny, nz))


def rade_marching_cubes(tsdf, weight, dims, origin, voxel: float, iso: float, workspace, verts,
                        max_verts: int, tris, max_tris: int, stream=None):
    """Returns (code, n_verts, n_tris); code is RADE_OK or RADE_ERR_CAPACITY
    (other errors raise).  Synchronises the stream."""
    nx, ny, nz = (int(d) for d in dims)
    o = (ctypes.c_double * 3)(*[float(x) for x in origin])
    nv, nt = ctypes.c_int64(0), ctypes.c_int64(0)
    ws_bytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    code = load().rade_marching_cubes(_p(tsdf), _p(weight), nx, ny, nz, o, float(voxel),
                                      float(iso), _p(workspace), ws_bytes, _p(verts),
                                      int(max_verts), _p(tris), int(max_tris), ctypes.byref(nv),
                                      ctypes.byref(nt), _stream(stream))
    if code not in (RADE_OK, RADE_ERR_CAPACITY):
        _check(code, "rade_marching_cubes")
    return code, nv.value, nt.value


def rade_marching_cubes_table():
    """(ntri uint8[256], tri uint8[256, 15]) compiled into the library."""
    ntri = np.zeros(256, np.uint8)
    tri = np.zeros((256, 15), np.uint8)
    _check(load().rade_marching_cubes_table(_p(ntri), _p(tri)), "rade_marching_cubes_table")
    return ntri, tri
