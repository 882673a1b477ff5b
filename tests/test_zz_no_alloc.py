"""fs_bin_noalloc (the bin stage with its scratch in the library's static
device buffer) against fs_bin with a caller workspace, through the C ABI.

Two calls in a row on one device, the second with a smaller input: the static
buffer keeps the first call's contents, so the second call shows that nothing
stale is read.  The first input has many scan partitions, the second one
footprints whose tiles the tile cache does not hold (the overflow queue in
the scratch buffer).  Keys, values and pair counts must be bit-identical.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

from paper_2604_10951_amd import _lib as L
from paper_2604_10951_amd import raster, scenes

pytestmark = pytest.mark.gpu


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _bin_both(scene, cams, tile, tile_mode="precise"):
    dev = torch.device("cuda:0")
    print(f"[case] noalloc bin: n={scene.n}, views={len(cams)}, tile={tile}, {tile_mode}", flush=True)
    rast = raster.Rasterizer(cams, tile=tile, tile_mode=tile_mode, device=dev)
    tens = raster.scene_tensors(scene, dev)
    fr = rast.render(*tens)                   # preprocess + sized buffers
    lib, b, n, V = rast.lib, rast._bufs, scene.n, rast.num_views
    m, s, q, o = tens[:4]
    stream = raster._stream(dev)
    cap = rast.capacity
    out = {}
    for name in ("ws", "noalloc"):
        keys = torch.full((cap,), -1, dtype=torch.int64, device=dev)
        vals = torch.full((cap,), -1, dtype=torch.int32, device=dev)
        cnt = torch.full((1,), -7, dtype=torch.int64, device=dev)
        P = ctypes.c_int64(-1)
        args = [_p(m), _p(s), _p(q), _p(o), n, _p(rast.cams_dev), V, ctypes.byref(rast.opts), _p(b["tiles"]),
                _p(b["tile_cache"]), _p(keys), _p(vals), cap, _p(cnt), ctypes.byref(P)]
        if name == "ws":
            st = lib.fs_bin(*args, _p(b["ws"]), stream)
        else:
            st = lib.fs_bin_noalloc(*args, stream)
        assert st == L.FS_OK, (name, st)
        torch.cuda.synchronize()
        out[name] = (int(P.value), int(cnt.item()), keys.cpu().numpy(), vals.cpu().numpy())
    Pw, Cw, kw, vw = out["ws"]
    Pn, Cn, kn, vn = out["noalloc"]
    assert Pw == Cw == Pn == Cn == fr.num_pairs > 0
    assert np.array_equal(kw[:Pw], kn[:Pn]), "keys differ"
    assert np.array_equal(vw[:Pw], vn[:Pn]), "values differ"
    assert np.all(kn[Pn:] == -1) and np.all(vn[Pn:] == -1), "writes past the pair count"
    return Pn


def test_noalloc_bin_matches_workspace_bin_on_two_calls():
    big, _ = scenes.topk_scene()                           # 300k surfels: 293 scan partitions
    cams = [scenes.centred_camera(640, 480), scenes.lookat_camera([0.3, -0.2, -1.0], [0, 0, 12], 320, 240)]
    p1 = _bin_both(big, cams, 8)
    needles, ncam = scenes.needle_scene()                  # 400 surfels, footprints re-derived in the overflow pass
    p2 = _bin_both(needles, [ncam], 16)
    assert p1 > p2
    print(f"noalloc bin: {p1} then {p2} pairs, bit-identical to the workspace bin", flush=True)


def test_noalloc_bin_bbox_mode_after_larger_call():
    scene, cam = scenes.parity_small()
    _bin_both(scene, [cam, scenes.centred_camera(96, 64)], 8, "bbox")
    _bin_both(scene.subset(np.arange(300)), [cam], 32, "bbox")


def test_noalloc_bin_rejects_inputs_beyond_its_scratch():
    dev = torch.device("cuda:0")
    lib = L.load()
    cam = scenes.centred_camera(64, 64)
    rast = raster.Rasterizer([cam, cam], tile=16, device=dev)
    small = torch.zeros(16, dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    n = L.FS_NOALLOC_MAX_RECORDS // 2 + 1                  # two views: one record over the limit
    st = lib.fs_bin_noalloc(_p(small), _p(small), _p(small), _p(small), n, _p(rast.cams_dev), 2,
                            ctypes.byref(rast.opts), _p(small), _p(small), None, None, 0, _p(cnt), None,
                            raster._stream(dev))
    assert st == L.FS_ERR_SCRATCH
    assert lib.fs_status_string(st) == b"input exceeds the static scratch buffer"
