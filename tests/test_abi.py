"""The C-ABI library loads and exports every symbol the header declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastsegsim.h")
LIB = os.path.join(ROOT, "paper_2604_10951_amd", "libfastsegsim.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_five_stages():
    syms = declared_symbols()
    for s in ("fs_preprocess", "fs_bin", "fs_sort", "fs_render_forward", "fs_render_backward"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(lib, s), s


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_host_only_entry_points_without_gpu():
    from paper_2604_10951_amd import _lib, scenes
    lib = _lib.load()
    cams = [scenes.centred_camera(640, 480), scenes.centred_camera(320, 240)]
    arr, tiles, pixels = _lib.make_cameras(cams, 16)
    assert tiles == 40 * 30 + 20 * 15 and pixels == 640 * 480 + 320 * 240
    assert arr[1].tile_offset == 1200 and arr[1].pixel_offset == 640 * 480
    o = _lib.make_opts()
    assert lib.fs_workspace_bytes(1000, 2, tiles, 10000, ctypes.byref(o)) > 0
    assert lib.fs_status_string(_lib.FS_ERR_CAPACITY) == b"pair capacity exceeded"
    bad = _lib.make_cameras.__globals__["FsCamera"] * 1
    a = bad()
    a[0].width, a[0].height = 0, 10
    assert lib.fs_layout_views(a, 1, 16, None, None) == _lib.FS_ERR_ARG
    # invalid options are rejected before anything touches a device
    o2 = _lib.make_opts(tile=12)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o2), None, None,
                             None, None) == _lib.FS_ERR_ARG
    o3 = _lib.make_opts(topk=-1)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o3), None, None,
                             None, None) == _lib.FS_ERR_ARG
    # the split render schedule exists for Top-K only
    o4 = _lib.make_opts(topk=0, schedule=_lib.FS_SCHED_SPLIT)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o4), None, None,
                             None, None) == _lib.FS_ERR_ARG
    o5 = _lib.make_opts(topk=8, schedule=_lib.FS_SCHED_SPLIT)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o5), None, None,
                             None, None) == _lib.FS_OK
    # Top-K modes: an unknown mode and a by-weight full blend are invalid
    o6 = _lib.make_opts(topk=8, schedule=_lib.FS_SCHED_SPLIT, topk_mode=2)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o6), None, None,
                             None, None) == _lib.FS_ERR_ARG
    o7 = _lib.make_opts(topk=0, topk_mode=_lib.FS_TOPK_WEIGHT)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o7), None, None,
                             None, None) == _lib.FS_ERR_ARG
    o8 = _lib.make_opts(topk=8, schedule=_lib.FS_SCHED_SPLIT, topk_mode=_lib.FS_TOPK_WEIGHT)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o8), None, None,
                             None, None) == _lib.FS_OK
    # tile modes 0-2 and the low-pass flag 0/1 only
    o9 = _lib.make_opts(topk=8, schedule=_lib.FS_SCHED_SPLIT, tile_mode=3)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o9), None, None,
                             None, None) == _lib.FS_ERR_ARG
    o10 = _lib.make_opts(topk=8, schedule=_lib.FS_SCHED_SPLIT, tile_mode=_lib.FS_TILES_LINEARISED, lowpass=1)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o10), None, None,
                             None, None) == _lib.FS_OK
    o11 = _lib.make_opts(topk=8, schedule=_lib.FS_SCHED_SPLIT, lowpass=2)
    assert lib.fs_preprocess(None, None, None, None, 0, ctypes.c_void_p(1), 1, ctypes.byref(o11), None, None,
                             None, None) == _lib.FS_ERR_ARG
    # the tile cache must be 16-byte aligned
    assert lib.fs_preprocess(ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 1,
                             ctypes.c_void_p(16), 1, ctypes.byref(o5), ctypes.c_void_p(16), ctypes.c_void_p(16),
                             ctypes.c_void_p(20), None) == _lib.FS_ERR_ARG
    # labels: the split schedule only, and every required output
    d = ctypes.c_void_p(256)
    og = _lib.make_opts(topk=8, schedule=_lib.FS_SCHED_GRID)
    assert lib.fs_render_labels(d, d, d, d, 16, 10, d, 1, 4, ctypes.byref(og), d, None, d, d, None, d,
                                None) == _lib.FS_ERR_UNSUPPORTED
    assert lib.fs_render_labels(d, d, d, d, 16, 10, d, 1, 4, ctypes.byref(o5), None, None, d, d, None, d,
                                None) == _lib.FS_ERR_ARG
    assert lib.fs_render_labels(d, d, d, d, 16, 10, d, 1, 4, ctypes.byref(o5), d, None, d, d, None, None,
                                None) == _lib.FS_ERR_ARG
    # instance labels: argument checks, and n == 0 enqueues nothing
    a16 = ctypes.c_void_p(4096)
    assert lib.fs_instance_labels(a16, 32, a16, 0, a16, a16, a16, 8, a16, None) == _lib.FS_OK
    assert lib.fs_instance_labels(a16, 32, a16, 10, a16, a16, a16, 65, a16, None) == _lib.FS_ERR_UNSUPPORTED
    assert lib.fs_instance_labels(a16, 6, a16, 10, a16, a16, a16, 8, a16, None) == _lib.FS_ERR_UNSUPPORTED
    assert lib.fs_instance_labels(a16, 32, a16, 10, a16, a16, a16, 0, a16, None) == _lib.FS_ERR_ARG
    assert lib.fs_instance_labels(ctypes.c_void_p(4100), 32, a16, 10, a16, a16, a16, 8, a16, None) == _lib.FS_ERR_ARG
    assert lib.fs_instance_labels(a16, 32, a16, 10, a16, a16, a16, 8, ctypes.c_void_p(4100), None) == _lib.FS_ERR_ARG
    assert lib.fs_instance_labels(a16, 32, None, 10, a16, a16, a16, 8, a16, None) == _lib.FS_ERR_ARG
