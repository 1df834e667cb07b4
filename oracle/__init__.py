"""FP64 CPU oracle of the RaDe-GS rasterizer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_2406_01467_amd``)
never does, and this package never imports the product.

The arithmetic lives in ``rade_oracle.cpp`` (plain C++17, FP64, OpenMP over
pixels); this module compiles it with g++ on first use and wraps it with
ctypes on NumPy arrays.

What each function follows (RaDe-GS, arXiv 2406.01467):

* :func:`project` -- Sec. 3.1 Eq. 1-2 (covariance, local affine projection),
  Sec. 3.2.2 Eq. 8-17 (ray space, q-hat by Eq. 13, p by Eq. 15-17), Sec. 3.3
  Eq. 21-22 (normal), spherical-harmonic colour (Sec. 3.1 under Eq. 3).
* :func:`render` -- Eq. 3 (front-to-back alpha blending) applied to colour,
  the per-pixel depth of Eq. 4, the normal of Eq. 22 and alpha; the median
  depth of Sec. 1.  Every pixel walks ALL Gaussians in (float32 depth, id)
  order.
* :func:`render_bwd`, :func:`project_bwd` -- the hand adjoint (pinned by
  central finite differences in the tests).
* :func:`bin_pairs` -- tile lists: (tile, depth) keys ordered by a stable sort.
* :func:`normal_consistency` -- Eq. 24 on the median-depth map.
* :func:`filter3d_var`, :func:`filter3d_apply` -- the 3D smoothing filter
  RaDe-GS trains with (Sec. 4.1).
* :func:`tsdf_fuse` (NumPy) and :func:`marching_cubes` (``mc.py``, NumPy
  plus a per-cell rule) -- mesh extraction from median-depth maps (Sec. 4.1).

Parity status: every function is pinned by the CPU tests in
``tests/test_oracle_*.py`` (closed forms, invariants, library routines, finite
differences), the tolerance helpers that set the GPU comparisons' floors and
exclusions included (:func:`gradient_error_scale`, the distortion's
``distortion_mag``, the magnitude bound of :func:`normal_consistency`, the
fragile-pixel flags: ``tests/test_oracle_tolerances.py``); nothing is "parity
unpinned" except the absolute agreement with the authors' unpublished CUDA
code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rade_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# Settings vector indices (mirror of the enum in rade_oracle.cpp).
S_DILATION, S_NEAR, S_ALPHA_MIN, S_ALPHA_MAX, S_T_MIN, S_POWER_CUT = 0, 1, 2, 3, 4, 5
S_FOV_CLAMP, S_DEGEN, S_BG, S_SH_DEGREE, S_TILE_W, S_TILE_H = 6, 7, 8, 11, 12, 13
S_FRAG_POWER, S_FRAG_ALPHA, S_FRAG_T, S_FRAG_MED, S_FRAG_CLAMP = 14, 15, 16, 17, 18
S_DEPTH_EXACT = 19
S_COUNT = 20

# Record fields (doubles per (view, Gaussian)).
R_FIELDS = ["uc", "vc", "z", "tc", "a", "b", "c", "o", "r", "g", "bl", "p0", "p1",
            "q0", "q1", "n0", "n1", "n2", "tau", "B00", "B01", "B11", "X", "Y",
            "ai00", "ai01", "ai02", "ai11", "ai12", "ai22"]
R = {k: i for i, k in enumerate(R_FIELDS)}
# Gradient fields of the projected quantities.
G_FIELDS = ["uc", "vc", "a", "b", "c", "o", "r", "g", "bl", "z", "p0", "p1", "n0", "n1", "n2"]
# Output fields per pixel.
O_FIELDS = ["r", "g", "b", "dexp", "dmed", "n0", "n1", "n2", "alpha", "tfinal", "dist",
            "dist_mag"]
# Upstream-gradient columns of render_bwd: colour 3, expected depth, median
# depth, normal 3, alpha, depth distortion (Eq. 23).
GOUT = 10

F_CULLED, F_VISIBLE, F_DEGENERATE, F_CLAMP_X, F_CLAMP_Y = 1, 2, 4, 8, 16
F_RGB_CLAMP = (32, 64, 128)


def build(force: bool = False) -> str:
    """Compile the oracle shared library with g++ (FP64, no FMA contraction)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
                   "-shared", _SRC, "-o", tmp]
            subprocess.check_call(cmd)
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_project.argtypes = [P, P, ctypes.c_int, ctypes.c_int64] + [P] * 8
        lib.oracle_render.argtypes = [P, P, ctypes.c_int64, P, P, P, ctypes.c_int64, P, P, P]
        lib.oracle_render_bwd.argtypes = [P, P, ctypes.c_int64, P, P, P, ctypes.c_int64, P, P, P]
        lib.oracle_project_bwd.argtypes = [P, P, ctypes.c_int, ctypes.c_int64] + [P] * 11
        lib.oracle_bin.argtypes = [P, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                   P, P, P, P, ctypes.c_int64, P]
        lib.oracle_bin.restype = ctypes.c_int64
        for f in ("oracle_settings_count", "oracle_view_count", "oracle_record_count",
                  "oracle_grad_count", "oracle_out_count"):
            getattr(lib, f).restype = ctypes.c_int
        assert lib.oracle_settings_count() == S_COUNT
        assert lib.oracle_record_count() == len(R_FIELDS)
        assert lib.oracle_grad_count() == len(G_FIELDS)
        assert lib.oracle_out_count() == len(O_FIELDS)
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def settings(sh_degree=0, dilation=0.3, near=0.2, alpha_min=1.0 / 255.0, alpha_max=0.99,
             t_min=1e-4, power_cut=4.5, fov_clamp=1.3, degenerate=1e-6, bg=(0.0, 0.0, 0.0),
             tile=(16, 16), frag_power=2e-5, frag_alpha=1e-5, frag_t=1e-4, frag_med=1e-5,
             frag_clamp=1e-5, depth_exact=False) -> np.ndarray:
    """Settings vector.  Defaults are the readings listed in the design notes:
    3DGS defaults for the quantities the paper leaves open."""
    s = np.zeros(S_COUNT, dtype=np.float64)
    s[S_DILATION], s[S_NEAR], s[S_ALPHA_MIN], s[S_ALPHA_MAX] = dilation, near, alpha_min, alpha_max
    s[S_T_MIN], s[S_POWER_CUT], s[S_FOV_CLAMP], s[S_DEGEN] = t_min, power_cut, fov_clamp, degenerate
    s[S_BG:S_BG + 3] = bg
    s[S_SH_DEGREE] = sh_degree
    s[S_TILE_W], s[S_TILE_H] = tile
    s[S_FRAG_POWER], s[S_FRAG_ALPHA], s[S_FRAG_T] = frag_power, frag_alpha, frag_t
    s[S_FRAG_MED], s[S_FRAG_CLAMP] = frag_med, frag_clamp
    s[S_DEPTH_EXACT] = 1.0 if depth_exact else 0.0
    return s


def view_vector(v) -> np.ndarray:
    """18 doubles: W, H, fx, fy, cx, cy, R (row-major), t."""
    out = np.zeros(18, dtype=np.float64)
    out[0], out[1] = v.width, v.height
    out[2], out[3] = np.float32(v.fx), np.float32(v.fy)
    out[4], out[5] = np.float32(v.cx), np.float32(v.cy)
    out[6:15] = np.asarray(v.R, dtype=np.float32).reshape(9)
    out[15:18] = np.asarray(v.t, dtype=np.float32).reshape(3)
    return out


def _scene_arrays(scene):
    c = np.ascontiguousarray
    return (c(scene.means, np.float32), c(scene.scales, np.float32), c(scene.quats, np.float32),
            c(scene.opacities, np.float32), c(scene.sh, np.float32))


def project(s: np.ndarray, views, scene):
    """Project a scene into views.  Returns (rec [V,N,24] f64, rect [V,N,4]
    int32, flags [V,N] int32)."""
    lib = _load()
    V, N = len(views), scene.n
    vv = np.ascontiguousarray(np.stack([view_vector(v) for v in views]))
    rec = np.zeros((V, N, len(R_FIELDS)), np.float64)
    rect = np.zeros((V, N, 4), np.int32)
    flags = np.zeros((V, N), np.int32)
    m, sc, q, o, sh = _scene_arrays(scene)
    lib.oracle_project(_ptr(s), _ptr(vv), V, N, _ptr(m), _ptr(sc), _ptr(q), _ptr(o), _ptr(sh),
                       _ptr(rec), _ptr(rect), _ptr(flags))
    return rec, rect, flags


def render(s: np.ndarray, view, rec: np.ndarray, flags: np.ndarray, pixels=None,
           want_sig: bool = False):
    """Render one view from its records (rec [N,24], flags [N]).  ``pixels``:
    optional int64 pixel indices (py*W + px).  Returns a dict of per-pixel
    arrays: color (n,3), depth_exp, depth_med, normal (n,3), alpha, t_final,
    count, last_id, median_id, fragile (bit 0: maps, bit 1: gradients), and
    optionally sig (discrete signature for finite-difference guards)."""
    lib = _load()
    N = rec.shape[0]
    rec = np.ascontiguousarray(rec, np.float64)
    flags = np.ascontiguousarray(flags, np.int32)
    vv = view_vector(view)
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int64)
    npix = view.width * view.height if pix is None else pix.shape[0]
    out = np.zeros((npix, len(O_FIELDS)), np.float64)
    iout = np.zeros((npix, 4), np.int64)
    sig = np.zeros(npix, np.uint64) if want_sig else None
    lib.oracle_render(_ptr(s), _ptr(vv), N, _ptr(rec), _ptr(flags), _ptr(pix), npix, _ptr(out),
                      _ptr(iout), _ptr(sig))
    res = dict(color=out[:, 0:3], depth_exp=out[:, 3], depth_med=out[:, 4], normal=out[:, 5:8],
               alpha=out[:, 8], t_final=out[:, 9], distortion=out[:, 10],
               distortion_mag=out[:, 11], count=iout[:, 0], last_id=iout[:, 1],
               median_id=iout[:, 2], fragile=iout[:, 3])
    if want_sig:
        res["sig"] = sig
    return res


def render_bwd(s: np.ndarray, view, rec: np.ndarray, flags: np.ndarray, gout: np.ndarray,
               pixels=None, gP: np.ndarray | None = None,
               gP_abs: np.ndarray | None = None) -> np.ndarray:
    """Adjoint of :func:`render`.  gout: (npix, 9) upstream gradients of
    (color 3, depth expected, depth median, normal 3, alpha), or (npix, 10)
    with the depth distortion of Eq. 23 last (its adjoint holds the blend
    weights constant, as the training loss detaches them).  Returns the
    gradient of the projected quantities, (N, 15) in the order of G_FIELDS.
    gP_abs, when given, accumulates over pixels a bound of the magnitudes of
    the quantities each per-pixel term is computed from (the same recursion
    run on absolute values): the round-off scale of those sums."""
    if s[S_DEPTH_EXACT]:
        raise NotImplementedError("the exact ray depth of Eq. 7 is a forward-only variant")
    lib = _load()
    N = rec.shape[0]
    vv = view_vector(view)
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int64)
    npix = view.width * view.height if pix is None else pix.shape[0]
    if gP is None:
        gP = np.zeros((N, len(G_FIELDS)), np.float64)
    if npix == 0:  # an empty pixel list contributes nothing
        return gP
    gout = np.asarray(gout, np.float64).reshape(npix, -1)
    if gout.shape[1] == 9:
        gout = np.concatenate([gout, np.zeros((npix, 1))], axis=1)
    gout = np.ascontiguousarray(gout).reshape(npix, GOUT)
    lib.oracle_render_bwd(_ptr(s), _ptr(vv), N, _ptr(np.ascontiguousarray(rec, np.float64)),
                          _ptr(np.ascontiguousarray(flags, np.int32)), _ptr(pix), npix,
                          _ptr(gout), _ptr(gP), _ptr(gP_abs))
    return gP


def project_bwd(s: np.ndarray, views, scene, gP: np.ndarray) -> dict:
    """Chain projected-quantity gradients gP [V,N,15] back to the parameters
    (summed over views)."""
    lib = _load()
    V, N = len(views), scene.n
    vv = np.ascontiguousarray(np.stack([view_vector(v) for v in views]))
    m, sc, q, o, sh = _scene_arrays(scene)
    out = dict(means=np.zeros((N, 3)), scales=np.zeros((N, 3)), quats=np.zeros((N, 4)),
               opacities=np.zeros(N), sh=np.zeros(sh.shape, np.float64))
    lib.oracle_project_bwd(_ptr(s), _ptr(vv), V, N, _ptr(m), _ptr(sc), _ptr(q), _ptr(o),
                           _ptr(sh), _ptr(np.ascontiguousarray(gP, np.float64)),
                           _ptr(out["means"]), _ptr(out["scales"]), _ptr(out["quats"]),
                           _ptr(out["opacities"]), _ptr(out["sh"]))
    return out


def bin_pairs(views, rect: np.ndarray, z: np.ndarray, tile=(16, 16)):
    """Binning reference.  rect [V,N,4] int32, z [V,N] float32.  Returns
    (ids uint32 [M], keys uint64 [M], ranges uint32 [sum tiles, 2])."""
    lib = _load()
    V, N = rect.shape[0], rect.shape[1]
    dims = np.ascontiguousarray([[v.width, v.height] for v in views], np.int32)
    tiles = sum(((v.width + tile[0] - 1) // tile[0]) * ((v.height + tile[1] - 1) // tile[1])
                for v in views)
    rect = np.ascontiguousarray(rect, np.int32)
    z = np.ascontiguousarray(z, np.float32)
    M = lib.oracle_bin(_ptr(dims), V, N, tile[0], tile[1], _ptr(rect), _ptr(z), None, None, 0,
                       None)
    ids = np.zeros(M, np.uint32)
    keys = np.zeros(M, np.uint64)
    ranges = np.zeros((tiles, 2), np.uint32)
    lib.oracle_bin(_ptr(dims), V, N, tile[0], tile[1], _ptr(rect), _ptr(z), _ptr(ids),
                   _ptr(keys), M, _ptr(ranges))
    return ids, keys, ranges


# ----------------------------------------------------------------------------
# Convenience: full forward / backward of a scene in views.

def forward(s: np.ndarray, views, scene, pixels=None, want_sig=False):
    rec, rect, flags = project(s, views, scene)
    outs = []
    for vi, v in enumerate(views):
        px = None if pixels is None else pixels[vi]
        outs.append(render(s, v, rec[vi], flags[vi], px, want_sig))
    return rec, rect, flags, outs


def backward(s: np.ndarray, views, scene, gouts, pixels=None, rec=None, flags=None) -> dict:
    """VJP of the whole path: gouts[v] is (npix_v, 9) or (npix_v, 10)."""
    if rec is None:
        rec, _, flags = project(s, views, scene)
    gP = np.zeros((len(views), scene.n, len(G_FIELDS)), np.float64)
    for vi, v in enumerate(views):
        px = None if pixels is None else pixels[vi]
        render_bwd(s, v, rec[vi], flags[vi], gouts[vi], px, gP[vi])
    return project_bwd(s, views, scene, gP)


def gradient_error_scale(s: np.ndarray, views, scene, gouts, pixels=None) -> dict:
    """Round-off scale of each parameter gradient element when the per-pixel
    terms are evaluated and summed in a reduced precision: for every
    projected quantity j of every view, the per-pixel magnitude bound of the
    adjoint recursion (absolute values throughout, so cancellation inside a
    term is accounted for) summed over pixels and pushed through
    |d parameter / d quantity_j|.  An evaluation whose elementary operations
    carry relative error u has |g - g_exact| <~ c u * scale with c of the
    order of the operation count."""
    rec, _, flags = project(s, views, scene)
    V, N = len(views), scene.n
    out = None
    for vi, v in enumerate(views):
        px = None if pixels is None else pixels[vi]
        gabs = np.zeros((N, len(G_FIELDS)), np.float64)
        render_bwd(s, v, rec[vi], flags[vi], gouts[vi], px, None, gabs)
        for j in range(len(G_FIELDS)):
            gP = np.zeros((1, N, len(G_FIELDS)), np.float64)
            gP[0, :, j] = gabs[:, j]
            r = project_bwd(s, [v], scene, gP)
            if out is None:
                out = {k: np.zeros_like(a) for k, a in r.items()}
            for k in r:
                out[k] += np.abs(r[k])
    return out


# ----------------------------------------------------------------------------
# Normal-consistency regulariser (Sec. 3.4, Eq. 24), FP64 NumPy.

def _abs_cross(a, b):
    """Componentwise bound |a x b| <= (|a_y b_z| + |a_z b_y|, ...)."""
    return np.stack([np.abs(a[1] * b[2]) + np.abs(a[2] * b[1]),
                     np.abs(a[2] * b[0]) + np.abs(a[0] * b[2]),
                     np.abs(a[0] * b[1]) + np.abs(a[1] * b[0])])


def normal_consistency(view, depth_med, normal, alpha, weight, magnitude=False):
    """Eq. 24 on the blended maps of one view: sum_i w_i (1 - n_i . n~) =
    alpha - N . n~ per pixel, averaged over interior pixels and scaled by
    ``weight``.  n~ is the unit normal of the back-projected median-depth map
    from central differences, oriented towards the camera (zero where the
    cross product vanishes).  depth_med (H,W), normal (3,H,W), alpha (H,W).
    Returns (loss, dL/d depth_med, dL/d normal, dL/d alpha); n~ is not
    detached."""
    D = np.asarray(depth_med, np.float64)
    Nm = np.asarray(normal, np.float64)
    A = np.asarray(alpha, np.float64)
    H, W = D.shape
    gD = np.zeros((H, W))
    gN = np.zeros((3, H, W))
    gA = np.zeros((H, W))
    if H < 3 or W < 3:
        return 0.0, gD, gN, gA
    fx, fy = float(np.float32(view.fx)), float(np.float32(view.fy))
    cx, cy = float(np.float32(view.cx)), float(np.float32(view.cy))
    xs = (np.arange(W) + 0.5 - cx) / fx
    ys = (np.arange(H) + 0.5 - cy) / fy
    r = np.stack([np.broadcast_to(xs[None, :], (H, W)), np.broadcast_to(ys[:, None], (H, W)),
                  np.ones((H, W))])
    P = D[None] * r                                   # back-projected points
    du = P[:, 1:-1, 2:] - P[:, 1:-1, :-2]             # central differences
    dv = P[:, 2:, 1:-1] - P[:, :-2, 1:-1]
    c = np.cross(du, dv, axis=0)
    nc = np.sqrt((c * c).sum(0))
    ok = nc > 0
    chat = np.where(ok, c / np.where(ok, nc, 1.0), 0.0)
    s = np.where((c * P[:, 1:-1, 1:-1]).sum(0) > 0, -1.0, 1.0)
    nt = s * chat
    Ni, Ai = Nm[:, 1:-1, 1:-1], A[1:-1, 1:-1]
    w = weight / ((H - 2) * (W - 2))
    loss = w * float((Ai - (Ni * nt).sum(0)).sum())
    gA[1:-1, 1:-1] = w
    gN[:, 1:-1, 1:-1] = -w * nt
    nd = (Ni * chat).sum(0)
    gc = np.where(ok, -w * s * (Ni - nd * chat) / np.where(ok, nc, 1.0), 0.0)
    g_du = np.cross(dv, gc, axis=0)
    g_dv = np.cross(gc, du, axis=0)
    gP = np.zeros((3, H, W))
    gP[:, 1:-1, 2:] += g_du
    gP[:, 1:-1, :-2] -= g_du
    gP[:, 2:, 1:-1] += g_dv
    gP[:, :-2, 1:-1] -= g_dv
    gD = (gP * r).sum(0)
    if not magnitude:
        return loss, gD, gN, gA
    # Round-off scale of dL/dD: the same recursion on magnitudes (the depth
    # gradient is a discrete divergence whose terms cancel on smooth maps).
    gc_m = np.where(ok, abs(w) * (np.abs(Ni) + np.abs(nd) * np.abs(chat)) /
                    np.where(ok, nc, 1.0), 0.0)
    gdu_m = _abs_cross(dv, gc_m)
    gdv_m = _abs_cross(gc_m, du)
    gP_m = np.zeros((3, H, W))
    gP_m[:, 1:-1, 2:] += gdu_m
    gP_m[:, 1:-1, :-2] += gdu_m
    gP_m[:, 2:, 1:-1] += gdv_m
    gP_m[:, :-2, 1:-1] += gdv_m
    gD_mag = (gP_m * np.abs(r)).sum(0)
    return loss, gD, gN, gA, gD_mag


# ----------------------------------------------------------------------------
# 3D smoothing filter (the Mip-Splatting filter the paper trains with,
# Sec. 4.1), FP64 NumPy.

def filter3d_var(views, means, near=0.2, scale=0.2, margin=0.15, return_fragile=False):
    """Per Gaussian: rate = max over views with camera z > near whose image,
    widened by margin x (width, height) on every side, holds the projected
    mean, of fx / z; variance scale / rate^2 (0 when no view sees the mean).
    With return_fragile, also flags means within 1e-6 px of a widened image
    border or within 1e-9 of the near plane (a decision FP rounding may flip)."""
    m = np.asarray(means, np.float32).astype(np.float64)
    best = np.zeros(m.shape[0])
    frag = np.zeros(m.shape[0], bool)
    for v in views:
        R = np.asarray(v.R, np.float32).astype(np.float64).reshape(3, 3)
        t = np.asarray(v.t, np.float32).astype(np.float64)
        fx, fy = float(np.float32(v.fx)), float(np.float32(v.fy))
        cx, cy = float(np.float32(v.cx)), float(np.float32(v.cy))
        x = m @ R.T + t
        z = x[:, 2]
        front = z > near
        zs = np.where(front, z, 1.0)
        u = fx * x[:, 0] / zs + cx
        w = fy * x[:, 1] / zs + cy
        mx, my = margin * v.width, margin * v.height
        inside = (u >= -mx) & (u <= v.width + mx) & (w >= -my) & (w <= v.height + my)
        ok = front & inside
        best = np.where(ok, np.maximum(best, fx / zs), best)
        edge = np.minimum.reduce([np.abs(u + mx), np.abs(u - v.width - mx), np.abs(w + my),
                                  np.abs(w - v.height - my)])
        frag |= (front & (edge < 1e-6)) | (np.abs(z - near) < 1e-9)
    var = np.where(best > 0, scale / np.where(best > 0, best, 1.0) ** 2, 0.0)
    return (var, frag) if return_fragile else var


def filter3d_apply(scales, opacities, var):
    """Filtered scales sqrt(s^2 + var) and opacities o sqrt(prod s^2 / prod
    (s^2 + var)) (the convolution keeps the Gaussian's integral)."""
    s = np.asarray(scales, np.float64)
    o = np.asarray(opacities, np.float64)
    f = np.asarray(var, np.float64)[:, None]
    t2 = s * s + f
    ratio = np.prod(np.where(t2 > 0, s * s / np.where(t2 > 0, t2, 1.0), 1.0), axis=1)
    return np.sqrt(t2), o * np.sqrt(ratio)


def filter3d_apply_bwd(scales, opacities, var, g_scales_f, g_opac_f):
    """Adjoint of filter3d_apply with var constant: d s_k = g_s'_k s_k / s'_k
    + g_o' o' var / (s_k s'_k^2), d o = g_o' sqrt(ratio)."""
    s = np.asarray(scales, np.float64)
    o = np.asarray(opacities, np.float64)
    f = np.asarray(var, np.float64)[:, None]
    gs = np.asarray(g_scales_f, np.float64)
    go = np.asarray(g_opac_f, np.float64)
    t2 = s * s + f
    sf = np.sqrt(t2)
    root = np.sqrt(np.prod(s * s / t2, axis=1))
    of = o * root
    ds = gs * s / sf + (go * of)[:, None] * f / (s * t2)
    return ds, go * root


# ----------------------------------------------------------------------------
# TSDF fusion of median-depth maps (Sec. 4.1, Mesh Extraction), FP64 NumPy.

def tsdf_fuse(views, depth_med, origin, voxel, dims, trunc, near=0.2, return_fragile=False):
    """Truncated signed distance of a voxel grid from per-view median-depth
    maps (depth_med[v]: (H, W)).  Voxel (i, j, k) has centre origin + (i +
    1/2, j + 1/2, k + 1/2) voxel and index (k ny + j) nx + i.  For every view
    with camera z > near whose projection of the centre falls in pixel
    (floor(u), floor(v)) of the image and whose median depth D there is
    positive (a surface): s = D - z; views with s >= -trunc contribute
    min(1, s / trunc) with weight 1.  Returns (tsdf = mean contribution, 0
    where none; weight = number of contributing views)."""
    nx, ny, nz = (int(d) for d in dims)
    o = np.asarray(origin, np.float64)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([o[0] + (ii.ravel() + 0.5) * voxel, o[1] + (jj.ravel() + 0.5) * voxel,
                  o[2] + (kk.ravel() + 0.5) * voxel], axis=1)
    F = np.zeros(X.shape[0])
    Wt = np.zeros(X.shape[0])
    frag = np.zeros(X.shape[0], bool)
    for v, D in zip(views, depth_med):
        R = np.asarray(v.R, np.float32).astype(np.float64).reshape(3, 3)
        t = np.asarray(v.t, np.float32).astype(np.float64)
        fx, fy = float(np.float32(v.fx)), float(np.float32(v.fy))
        cx, cy = float(np.float32(v.cx)), float(np.float32(v.cy))
        x = X @ R.T + t
        z = x[:, 2]
        front = z > near
        zs = np.where(front, z, 1.0)
        u = fx * x[:, 0] / zs + cx
        w = fy * x[:, 1] / zs + cy
        px, py = np.floor(u), np.floor(w)
        inside = front & (px >= 0) & (px < v.width) & (py >= 0) & (py < v.height)
        pxi = np.where(inside, px, 0).astype(np.int64)
        pyi = np.where(inside, py, 0).astype(np.int64)
        d = np.asarray(D, np.float64)[pyi, pxi]
        s = d - z
        ok = inside & (d > 0) & (s >= -trunc)
        F += np.where(ok, np.minimum(1.0, s / trunc), 0.0)
        Wt += ok
        # decisions rounding may flip: a centre on a pixel border, the
        # truncation edge, the near plane
        frag |= front & ((np.abs(u - np.round(u)) < 1e-7) | (np.abs(w - np.round(w)) < 1e-7))
        frag |= inside & (d > 0) & (np.abs(s + trunc) < 1e-5 * (1.0 + abs(trunc)))
        frag |= np.abs(z - near) < 1e-9
    tsdf = np.where(Wt > 0, F / np.where(Wt > 0, Wt, 1.0), 0.0)
    return (tsdf, Wt, frag) if return_fragile else (tsdf, Wt)


from .mc import cell_triangles, marching_cubes  # noqa: E402,F401  (Sec. 4.1, Marching Cubes)
