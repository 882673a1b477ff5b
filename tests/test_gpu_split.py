"""Split Top-K schedule (selection pass + gather pass).  The selection pass
takes the same per-pixel decisions with the same arithmetic as the fused
renderer and the gather pass adds the same products in the same order, so
every output must be bit-identical to the fused kernel's, for every channel
count (vector and scalar row paths, several channel vectors per thread),
feature storage type, tile size and view layout; the oracle checks are in the
parity tests."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2604_10951_amd import raster, scenes
from tests.test_gpu_parity import check_image

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


def _case(name):
    print(f"[case] {name}", flush=True)


def _frame(cams, tens, **kw):
    rast = raster.Rasterizer(cams, device=_dev(), **kw)
    fr = rast.render(*tens, want_last=True, want_idx=True)
    torch.cuda.synchronize()
    return rast, fr


def _same(a, b):
    for name in ("feat", "T", "n", "last", "idx"):
        x, y = getattr(a, name), getattr(b, name)
        assert torch.equal(x, y), name


@pytest.mark.parametrize("C_extra,tile,K,dtype", [
    (16, 8, 8, "f32"),     # C = 19: scalar rows
    (61, 8, 5, "f32"),     # C = 64: float4 rows, 16 threads per pixel
    (125, 16, 8, "f32"),   # C = 128: 32 threads per pixel
    (297, 32, 3, "f32"),   # C = 300: 64 threads per pixel, two vectors each
    (125, 8, 8, "bf16"),   # C = 128 bfloat16: 8-element vectors
    (17, 16, 4, "bf16"),   # C = 20 bfloat16: scalar rows
    (61, 8, 64, "f32"),    # K = 64
])
def test_split_bit_identical_to_fused(C_extra, tile, K, dtype):
    _case(f"split C={C_extra + 3} tile={tile} K={K} {dtype}")
    scene = scenes.uniform_scene(2500, seed=21, feat_channels=C_extra)
    cams = [scenes.centred_camera(101, 77), scenes.lookat_camera([0.4, -0.2, -1.0], [0, 0, 4], 80, 72)]
    tens = raster.scene_tensors(scene, _dev(), dtype)
    _, a = _frame(cams, tens, tile=tile, topk=K, feat_dtype=dtype, schedule="grid")
    _, b = _frame(cams, tens, tile=tile, topk=K, feat_dtype=dtype, schedule="split")
    assert int(a.n.sum()) > 1000
    _same(a, b)


def test_split_workload_full_image_and_counters():
    """300k clustered surfels, 640x480, C = 64, K = 8 against the oracle;
    at 8x8 tiles both schedules count the same needed rows, blends and
    blocks.  Walked entries are counted per staged batch, and the two
    schedules stage batches of different sizes, so only their bound is
    common."""
    _case("split 300k")
    scene, cam = scenes.topk_scene()
    tens = raster.scene_tensors(scene, _dev())
    got = []
    for schedule in ("grid", "split"):
        rast = raster.Rasterizer(cam, tile=8, topk=8, schedule=schedule, device=_dev())
        fr = rast.render(*tens, want_idx=True)
        counters = torch.zeros(4, dtype=torch.int64, device=_dev())
        rast.render_forward(tens[4], counters=counters)
        torch.cuda.synchronize()
        got.append(counters.cpu().numpy())
    assert np.array_equal(got[0][1:], got[1][1:]), got
    assert got[0][0] >= got[0][1] and got[1][0] >= got[1][1], got
    c = got[1]
    assert c[2] == int(fr.n.sum()) and c[3] == rast.total_tiles and c[0] >= c[1] > 0
    ref = oracle.render_scene(scene, cam, K=8, kcap=8)
    check_image(fr, ref, rast, 0, scene.channels, 8, "split 300k")


def test_split_rejects_full_blend():
    with pytest.raises(Exception):
        _frame([scenes.centred_camera(16, 16)],
               raster.scene_tensors(scenes.uniform_scene(10, seed=1), _dev()), tile=8, topk=0, schedule="split")


@pytest.mark.parametrize("K,dtype,C_extra", [(8, "f32", 125), (16, "f32", 125), (16, "bf16", 253)])
def test_split_many_rows_per_block(K, dtype, C_extra):
    """Dense small surfels: every pixel blends K different surfels, so a block
    needs far more feature rows than one staged window holds."""
    _case(f"split dense K={K} {dtype} C={C_extra + 3}")
    scene = scenes.uniform_scene(40000, seed=4, scale_range=(0.003, 0.01), feat_channels=C_extra)
    cam = scenes.centred_camera(64, 48)
    tens = raster.scene_tensors(scene, _dev(), dtype)
    _, a = _frame([cam], tens, tile=8, topk=K, feat_dtype=dtype, schedule="grid")
    rast, b = _frame([cam], tens, tile=8, topk=K, feat_dtype=dtype, schedule="split")
    counters = torch.zeros(4, dtype=torch.int64, device=_dev())
    rast.render_forward(tens[4], counters=counters)
    torch.cuda.synchronize()
    rows, blocks = int(counters[1]), int(counters[3])
    assert rows > 100 * blocks, (rows, blocks)   # windows of at most 64 rows
    _same(a, b)
