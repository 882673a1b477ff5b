"""ctypes binding of libfastsegsim.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/fastsegsim.h with
the same name; no arithmetic of the method happens in Python.  Loading fails
loudly if the HIP library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastsegsim.so")

FS_OK, FS_ERR_ARG, FS_ERR_CAPACITY, FS_ERR_HIP, FS_ERR_UNSUPPORTED, FS_ERR_SCRATCH = 0, 1, 2, 3, 4, 5
FS_NOALLOC_MAX_RECORDS = 4194304
FS_TILES_PRECISE, FS_TILES_BBOX, FS_TILES_LINEARISED = 0, 1, 2
FS_FEAT_F32, FS_FEAT_BF16 = 0, 1
FS_SCHED_GRID, FS_SCHED_PERSISTENT, FS_SCHED_SPLIT = 0, 1, 2
FS_TOPK_FIRST, FS_TOPK_WEIGHT = 0, 1
FS_RECORD_BYTES = 96
FS_TILE_CACHE_WORDS = 4
FS_GRAD_RECORD_FLOATS = 12


class FsCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("z_near", ctypes.c_float),
                ("tile_offset", ctypes.c_int32), ("pixel_offset", ctypes.c_int64)]


class FsOpts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("topk", ctypes.c_int32), ("tile_mode", ctypes.c_int32),
                ("feat_dtype", ctypes.c_int32), ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("t_stop", ctypes.c_float), ("batch", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("topk_mode", ctypes.c_int32), ("lowpass", ctypes.c_int32)]


assert ctypes.sizeof(FsCamera) == 88
assert ctypes.sizeof(FsOpts) == 44


class FastSegSimError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = _lib_or_none().fs_status_string(status).decode() if _lib_or_none() else str(status)
        extra = ""
        if status == FS_ERR_HIP and _lib_or_none():
            extra = f" (hipError {_lib_or_none().fs_last_hip_error()})"
        super().__init__(f"{what}: {msg}{extra}")


_lib = None

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32

# exported symbols and their argument types
SIGNATURES = {
    "fs_layout_views": ([ctypes.POINTER(FsCamera), I32, I32, ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
    "fs_workspace_bytes": ([I64, I32, I64, I64, ctypes.POINTER(FsOpts)], ctypes.c_size_t),
    "fs_preprocess": ([P, P, P, P, I64, P, I32, ctypes.POINTER(FsOpts), P, P, P, P], I32),
    "fs_bin": ([P, P, P, P, I64, P, I32, ctypes.POINTER(FsOpts), P, P, P, P, I64, P, ctypes.POINTER(I64), P, P], I32),
    "fs_bin_noalloc": ([P, P, P, P, I64, P, I32, ctypes.POINTER(FsOpts), P, P, P, P, I64, P, ctypes.POINTER(I64), P],
                       I32),
    "fs_sort": ([P, P, I64, P, I64, I64, P, P, P], I32),
    "fs_render_forward": ([P, P, P, P, P, I32, I64, P, I32, I64, ctypes.POINTER(FsOpts), P, P, P, P, P, P, P, P, P,
                           P], I32),
    "fs_render_labels": ([P, P, P, P, I32, I64, P, I32, I64, ctypes.POINTER(FsOpts), P, P, P, P, P, P, P], I32),
    "fs_instance_labels": ([P, I32, P, I64, P, P, P, I32, P, P], I32),
    "fs_render_backward": ([P, P, P, P, P, P, P, P, I32, I64, P, I32, I64, ctypes.POINTER(FsOpts), P, P, P, P, P, P,
                            P, P, P, P, P, P], I32),
    "fs_status_string": ([I32], ctypes.c_char_p),
    "fs_last_hip_error": ([], I32),
}


def _lib_or_none():
    return _lib


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build the HIP library first (python -c 'import __graft_entry__ as g; "
                          "g.build()')")
    lib = ctypes.CDLL(path)
    for name, (argtypes, restype) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = restype
    _lib = lib
    return lib


def check(status: int, what: str) -> None:
    if status != FS_OK:
        raise FastSegSimError(status, what)


def make_opts(tile: int = 16, topk: int = 0, tile_mode: int = FS_TILES_PRECISE, feat_dtype: int = FS_FEAT_F32,
              alpha_min: float = 1.0 / 255.0, alpha_max: float = 0.99, t_stop: float = 1e-4,
              batch: int = 0, schedule: int = FS_SCHED_GRID, topk_mode: int = FS_TOPK_FIRST,
              lowpass: int = 0) -> FsOpts:
    return FsOpts(tile, topk, tile_mode, feat_dtype, alpha_min, alpha_max, t_stop, batch, schedule, topk_mode,
                  lowpass)


def make_cameras(cams, tile: int):
    """Pack cameras into an fs_camera array laid out by fs_layout_views.

    Returns (array, total_tiles, total_pixels)."""
    lib = load()
    arr = (FsCamera * len(cams))()
    for i, c in enumerate(cams):
        a = arr[i]
        a.width, a.height = int(c.width), int(c.height)
        a.fx, a.fy, a.cx, a.cy = c.fx, c.fy, c.cx, c.cy
        R = [float(x) for x in c.R.reshape(9)]
        t = [float(x) for x in c.t.reshape(3)]
        for j in range(9):
            a.R[j] = R[j]
        for j in range(3):
            a.t[j] = t[j]
        a.z_near = c.z_near
    tt, tp = I64(0), I64(0)
    check(lib.fs_layout_views(arr, len(cams), tile, ctypes.byref(tt), ctypes.byref(tp)), "fs_layout_views")
    return arr, int(tt.value), int(tp.value)
