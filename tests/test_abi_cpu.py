"""CPU checks of the C ABI: the library loads, exports every function that
include/rade.h declares, the header is valid C with the documented struct
sizes, and invalid arguments are rejected on the host before any launch."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rade.h")


def _lib():
    from paper_2406_01467_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2406_01467_amd import build
        build.build()
    return _lib


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(rade_\w+)\s*\(", text,
                                 re.M)))


def test_exports_every_declared_symbol():
    lib = _lib()
    names = _declared()
    assert len(names) == 25, names
    so = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(so, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (rade_\w+)", out))
    assert set(names) <= exported
    assert set(lib.EXPORTED) == set(names)


def test_header_is_c_and_struct_sizes(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "rade.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   "int main(void){printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(rade_settings),"
                   " sizeof(rade_view), sizeof(rade_splat), offsetof(rade_splat, rect),"
                   " offsetof(rade_view, pix_offset)); return 0;}\n")
    exe = tmp_path / "t"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I",
                           os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    sizes = subprocess.check_output([str(exe)]).decode().split()
    assert sizes == ["120", "96", "80", "72", "80"]
    lib = _lib()
    assert ctypes.sizeof(lib.CSettings) == 120 and ctypes.sizeof(lib.CView) == 96
    assert lib.SPLAT_DTYPE.itemsize == 80 and lib.SPLAT_DTYPE.fields["rect"][1] == 72


def test_views_prepare_offsets():
    lib = _lib()
    import synth
    views = [synth.identity_view(100, 70), synth.identity_view(33, 17), synth.identity_view(16, 16)]
    vc = lib.make_views(views)
    P, T = lib.rade_views_prepare(lib.Settings(tile_w=16, tile_h=16), vc)
    assert P == 100 * 70 + 33 * 17 + 256
    assert [vc[i].tiles_x for i in range(3)] == [7, 3, 1]
    assert [vc[i].tiles_y for i in range(3)] == [5, 2, 1]
    assert [vc[i].pix_offset for i in range(3)] == [0, 7000, 7000 + 561]
    assert [vc[i].tile_offset for i in range(3)] == [0, 35, 41]
    assert T == 42
    P2, T2 = lib.rade_views_prepare(lib.Settings(tile_w=32, tile_h=16), vc)
    assert T2 == 4 * 5 + 2 * 2 + 1 and vc[0].tiles_x == 4


@pytest.mark.parametrize("bad", [dict(tile_w=12), dict(tile_h=64), dict(sh_degree=4), dict(schedule=3),
                                 dict(alpha_min=0.0), dict(t_min=1.5), dict(power_cut=-1.0),
                                 # the backward divides by 1 - alpha: the clamp must stay
                                 # below 1, also after rounding to FP32
                                 dict(alpha_max=1.0), dict(alpha_max=1.0 - 1e-9),
                                 dict(depth_mode=3), dict(wave_w=12), dict(batch=96),
                                 dict(tile_w=8, tile_h=8, wave_w=16),
                                 dict(tile_w=16, tile_h=32, wave_w=32)])
def test_invalid_settings_rejected_without_launch(bad):
    lib = _lib()
    import synth
    vc = lib.make_views([synth.identity_view(32, 32)])
    with pytest.raises(lib.RadeError) as ei:
        lib.rade_views_prepare(lib.Settings(**bad), vc)
    assert ei.value.code == lib.RADE_ERR_INVALID_ARG
    # rade_project validates before touching the device: NULL pointers with
    # an invalid setting or a zero view count never reach HIP
    so = lib.load()
    s = lib.Settings(**bad).c()
    assert so.rade_project(ctypes.byref(s), None, 1, 10, *([None] * 9), None) == \
        lib.RADE_ERR_INVALID_ARG


def test_null_pointers_rejected():
    lib = _lib()
    so = lib.load()
    s = lib.Settings().c()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert so.rade_project(ctypes.byref(s), dummy, 1, 10, None, dummy, dummy, dummy, dummy,
                           dummy, dummy, None, None, None) == lib.RADE_ERR_INVALID_ARG
    assert so.rade_project(ctypes.byref(s), dummy, 0, 10, *([dummy] * 9), None) == \
        lib.RADE_ERR_INVALID_ARG
    # misaligned quaternion array, misaligned binning records
    assert so.rade_project(ctypes.byref(s), dummy, 1, 10, dummy, dummy, ctypes.c_void_p(20),
                           dummy, dummy, dummy, dummy, None, None, None) == lib.RADE_ERR_INVALID_ARG
    assert so.rade_project(ctypes.byref(s), dummy, 1, 10, *([dummy] * 7), ctypes.c_void_p(24),
                           None, None) == lib.RADE_ERR_INVALID_ARG
    # exact depth: the depth_quad records are required and 16-byte aligned;
    # the backward rejects the mode; unknown modes and lane_masks values
    # other than 0 and 1 are rejected
    se = lib.Settings(depth_mode=lib.RADE_DEPTH_EXACT).c()
    assert so.rade_project(ctypes.byref(se), dummy, 1, 10, *([dummy] * 7), None, None, None) == \
        lib.RADE_ERR_INVALID_ARG
    assert so.rade_project(ctypes.byref(se), dummy, 1, 10, *([dummy] * 7), None,
                           ctypes.c_void_p(24), None) == lib.RADE_ERR_INVALID_ARG
    bad = lib.Settings(depth_mode=2).c()
    assert so.rade_project(ctypes.byref(bad), dummy, 1, 10, *([dummy] * 9), None) == \
        lib.RADE_ERR_INVALID_ARG
    res = lib.Settings().c()
    res.lane_masks = 2
    assert so.rade_project(ctypes.byref(res), dummy, 1, 10, *([dummy] * 9), None) == \
        lib.RADE_ERR_INVALID_ARG
    import synth
    vc = lib.make_views([synth.identity_view(32, 32)])
    lib.rade_views_prepare(lib.Settings(), vc)
    # workspace too small -> RADE_ERR_WORKSPACE before any launch
    code = so.rade_bin_sort(ctypes.byref(s), vc, dummy, 1, 10, dummy, dummy, dummy, dummy, None,
                            100, dummy, None, dummy, 1, None)
    assert code == lib.RADE_ERR_WORKSPACE
    # views not prepared for this tile size
    s2 = lib.Settings(tile_w=8, tile_h=8).c()
    code = so.rade_bin_sort(ctypes.byref(s2), vc, dummy, 1, 10, dummy, dummy, dummy, dummy, None,
                            100, dummy, None, dummy, 1 << 30, None)
    assert code == lib.RADE_ERR_INVALID_ARG
    # the binning records are required and 16-byte aligned
    for brec in (None, ctypes.c_void_p(24)):
        code = so.rade_bin_sort(ctypes.byref(s), vc, dummy, 1, 10, dummy, brec, dummy, dummy,
                                None, 100, dummy, None, dummy, 1 << 30, None)
        assert code == lib.RADE_ERR_INVALID_ARG
    assert lib.strerror(lib.RADE_ERR_CAPACITY).startswith("output capacity")


def test_workspace_sizes_monotone():
    lib = _lib()
    a = lib.rade_bin_sort_workspace(1, 1000, 5000, 64)
    b = lib.rade_bin_sort_workspace(1, 1000, 50000, 64)
    c = lib.rade_bin_sort_workspace(2, 1000, 5000, 64)
    assert 0 < a < b and a < c
    s = lib.Settings()
    assert lib.rade_render_bwd_workspace(s, 1, 1000, False) >= 1000 * 64
    assert lib.rade_render_bwd_workspace(s, 1, 1000, True) >= 1000 * (64 + 80)


def test_marching_cubes_table_matches_the_oracle_rule():
    """The table compiled into the library (generated at compile time from
    the face rule) equals the oracle's per-code triangulation, triangle for
    triangle, for all 256 cell codes."""
    import oracle
    lib = _lib()
    ntri, tri = lib.rade_marching_cubes_table()
    for code in range(256):
        want = oracle.cell_triangles(code)
        assert ntri[code] == len(want), code
        got = [tuple(int(x) for x in tri[code, 3 * t: 3 * t + 3]) for t in range(ntri[code])]
        assert got == [tuple(t) for t in want], code


def test_marching_cubes_rejects_bad_arguments_on_the_host():
    lib = _lib()
    so = lib.load()
    f = np.zeros(8, np.float32)
    ws = np.zeros(1 << 16, np.uint8)
    out_v = np.zeros(30, np.float32)
    out_t = np.zeros(30, np.uint32)
    nv, nt = ctypes.c_int64(0), ctypes.c_int64(0)
    o = (ctypes.c_double * 3)(0.0, 0.0, 0.0)

    def call(dims=(2, 2, 2), voxel=0.1, iso=0.0, ws_bytes=ws.nbytes, origin=o, max_v=10):
        return so.rade_marching_cubes(f.ctypes.data, f.ctypes.data, *dims, origin, voxel, iso,
                                      ws.ctypes.data, ws_bytes, out_v.ctypes.data, max_v,
                                      out_t.ctypes.data, 10, ctypes.byref(nv), ctypes.byref(nt),
                                      None)
    assert call(dims=(0, 2, 2)) == lib.RADE_ERR_INVALID_ARG
    assert call(dims=(2048, 2048, 1024)) == lib.RADE_ERR_INVALID_ARG   # 32-bit vertex ids
    assert call(voxel=0.0) == lib.RADE_ERR_INVALID_ARG
    assert call(voxel=float("inf")) == lib.RADE_ERR_INVALID_ARG
    assert call(iso=float("nan")) == lib.RADE_ERR_INVALID_ARG
    assert call(origin=(ctypes.c_double * 3)(0.0, float("nan"), 0.0)) == lib.RADE_ERR_INVALID_ARG
    assert call(max_v=-1) == lib.RADE_ERR_INVALID_ARG
    assert call(ws_bytes=16) == lib.RADE_ERR_WORKSPACE
    assert lib.rade_marching_cubes_workspace((2, 2, 2)) <= ws.nbytes
    assert lib.rade_marching_cubes_workspace((0, 1, 1)) == 0


def test_render_bwd_rejects_a_misaligned_workspace():
    """The gradient records in the workspace move in 16-byte words: a
    workspace that is not 16-byte aligned is rejected before any launch
    (the device pointers here are never dereferenced)."""
    lib = _lib()
    import synth
    so = lib.load()
    s = lib.Settings()
    vc = lib.make_views([synth.identity_view(32, 32)])
    lib.rade_views_prepare(s, vc)
    d = ctypes.c_void_p(256)
    head = [ctypes.byref(s.c()), vc, d, 1, 10] + [d] * 5 + [d, d, d, d, d, d, d] + [d] * 4 + \
        [None, None, None]
    args = head + [None] + [d] * 5  # no lane-mask cache
    big = 1 << 30
    assert so.rade_render_bwd(*args, ctypes.c_void_p(256 + 4), big, None) == \
        lib.RADE_ERR_INVALID_ARG
    assert so.rade_render_bwd(*args, None, big, None) == lib.RADE_ERR_WORKSPACE
    # a lane-mask cache is read in 16-byte words: misaligned is rejected too
    assert so.rade_render_bwd(*(head + [ctypes.c_void_p(256 + 8)] + [d] * 5), d, big, None) == \
        lib.RADE_ERR_INVALID_ARG


def test_render_fwd_rejects_a_misaligned_lane_mask_cache():
    """The forward writes the lane-mask cache in 16-byte words: a pointer that
    is not 16-byte aligned is rejected before the device check (the dummy
    device pointers are never dereferenced); NULL means no cache."""
    lib = _lib()
    import synth
    so = lib.load()
    s = lib.Settings()
    vc = lib.make_views([synth.identity_view(32, 32)])
    lib.rade_views_prepare(s, vc)
    d = ctypes.c_void_p(256)
    head = [ctypes.byref(s.c()), vc, d, 1, 10, d, d, d, None] + [d] * 7 + [None] * 4
    assert so.rade_render_fwd(*head, ctypes.c_void_p(256 + 8), None) == lib.RADE_ERR_INVALID_ARG
    if _no_gpu():
        assert so.rade_render_fwd(*head, None, None) == lib.RADE_ERR_UNSUPPORTED_DEVICE
        assert so.rade_render_fwd(*head, d, None) == lib.RADE_ERR_UNSUPPORTED_DEVICE


def test_lane_mask_bytes_follow_the_launch_shape():
    """8 bytes per (pair, 8x8 wave) where the launch shape keeps lane masks
    (8x8 tiles of 8x8 waves; lane_masks = 1 on larger tiles of 8x8 waves with
    one splat staged per thread), 0 elsewhere and for invalid arguments."""
    lib = _lib()

    def nbytes(n, **kw):
        return lib.rade_lane_mask_bytes(lib.Settings(**kw), n)

    assert nbytes(1000, tile_w=16, tile_h=16) == 0
    assert nbytes(1000, tile_w=16, tile_h=16, lane_masks=1) == 1000 * 4 * 8
    assert nbytes(1000, tile_w=32, tile_h=16, lane_masks=1) == 1000 * 8 * 8
    assert nbytes(1000, tile_w=16, tile_h=8, lane_masks=1) == 1000 * 2 * 8
    assert nbytes(1000, tile_w=16, tile_h=16, lane_masks=1, batch=128) == 0
    assert nbytes(1000, tile_w=16, tile_h=16, lane_masks=1, wave_w=16) == 0
    assert nbytes(1000, tile_w=8, tile_h=8) == 1000 * 8
    assert nbytes(1000, tile_w=8, tile_h=8, batch=256) == 1000 * 8
    assert nbytes(0, tile_w=8, tile_h=8) == 0
    assert nbytes(-1, tile_w=8, tile_h=8) == 0
    assert nbytes(1000, tile_w=16, tile_h=16, lane_masks=2) == 0


def _no_gpu() -> bool:
    import torch
    return not torch.cuda.is_available()


def test_error_codes_are_distinct():
    lib = _lib()
    codes = [lib.RADE_ERR_INVALID_ARG, lib.RADE_ERR_CAPACITY, lib.RADE_ERR_HIP,
             lib.RADE_ERR_UNSUPPORTED_DEVICE, lib.RADE_ERR_WORKSPACE, lib.RADE_ERR_TOO_LARGE]
    assert len(set(codes)) == len(codes) and lib.RADE_OK not in codes
    assert lib.RADE_ERR_UNSUPPORTED_DEVICE == -4 and lib.RADE_ERR_WORKSPACE == -5
    assert lib.RADE_ERR_TOO_LARGE == -6
    msgs = {lib.strerror(c) for c in codes}
    assert len(msgs) == len(codes) and "gfx950" in lib.strerror(lib.RADE_ERR_UNSUPPORTED_DEVICE)


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device path")
def test_no_device_is_unsupported_and_nothing_launches():
    """Without a gfx950 device (here: none at all) every call whose arguments
    are valid stops at the device check with RADE_ERR_UNSUPPORTED_DEVICE,
    after argument validation and before any launch (the dummy device
    pointers are never dereferenced); invalid arguments still report
    RADE_ERR_INVALID_ARG first."""
    lib = _lib()
    import synth
    so = lib.load()
    assert lib.rade_device_check() == lib.RADE_ERR_UNSUPPORTED_DEVICE
    assert lib.rade_device_check() == lib.RADE_ERR_UNSUPPORTED_DEVICE  # cached answer
    s = lib.Settings().c()
    d = ctypes.c_void_p(256)
    assert so.rade_project(ctypes.byref(s), d, 1, 10, *([d] * 7), None, None, None) == \
        lib.RADE_ERR_UNSUPPORTED_DEVICE
    assert so.rade_project(ctypes.byref(s), d, 0, 10, *([d] * 7), None, None, None) == \
        lib.RADE_ERR_INVALID_ARG
    vc = lib.make_views([synth.identity_view(32, 32)])
    lib.rade_views_prepare(lib.Settings(), vc)
    assert so.rade_render_fwd(ctypes.byref(s), vc, d, 1, 10, d, d, d, None, *([d] * 7),
                              None, None, None, None, None, None) == \
        lib.RADE_ERR_UNSUPPORTED_DEVICE
    ws = lib.rade_bin_sort_workspace(1, 10, 100, 4)
    assert so.rade_bin_sort(ctypes.byref(s), vc, d, 1, 10, d, d, d, d, None, 100, d, None, d,
                            ws, None) == lib.RADE_ERR_UNSUPPORTED_DEVICE
    assert so.rade_filter3d_apply(10, d, d, d, d, d, None) == lib.RADE_ERR_UNSUPPORTED_DEVICE


def test_noalloc_limit_is_checked_on_the_host():
    """The allocation-free Eq. 24 entry point rejects views with more 32x8
    blocks than its fixed scratch holds, before the device check and before
    anything is enqueued (the dummy pointers are never dereferenced); the
    header's limit is the binding's."""
    lib = _lib()
    import synth
    so = lib.load()
    text = open(HEADER).read()
    m = re.search(r"#define RADE_NC_NOALLOC_MAX_BLOCKS (\d+)", text)
    assert m and int(m.group(1)) == lib.RADE_NC_NOALLOC_MAX_BLOCKS
    d = ctypes.c_void_p(256)

    def call(sizes):
        vc = lib.make_views([synth.identity_view(w, h) for w, h in sizes])
        lib.rade_views_prepare(lib.Settings(), vc)
        return so.rade_normal_consistency_noalloc(vc, d, len(sizes), d, d, d,
                                                  ctypes.c_float(1.0), d, d, d, d, 1, None)
    # 128 x 512 blocks per 4096 x 4096 view: two fill the scratch exactly
    assert call([(8192, 8192)]) == lib.RADE_ERR_TOO_LARGE
    assert call([(4096, 4096), (4096, 4096), (32, 8)]) == lib.RADE_ERR_TOO_LARGE
    ok = lib.RADE_ERR_UNSUPPORTED_DEVICE if _no_gpu() else None
    if ok is not None:
        assert call([(4096, 4096), (4096, 4096)]) == ok
        assert call([(31, 9)]) == ok
    vc = lib.make_views([synth.identity_view(32, 8)])
    lib.rade_views_prepare(lib.Settings(), vc)
    assert so.rade_normal_consistency_noalloc(vc, d, 1, d, None, d, ctypes.c_float(1.0), d, d, d,
                                              d, 1, None) == lib.RADE_ERR_INVALID_ARG
