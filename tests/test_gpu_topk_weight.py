"""Top-K by weight (the alternative reading of Sec. 3.4; the split schedule's
FS_TOPK_WEIGHT mode) against the oracle: the K contributors of largest
weight alpha T of each pixel's full walk, blended front to back."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2604_10951_amd import _lib, raster, scenes
from tests.test_gpu_parity import check_image

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


def _case(name):
    print(f"[case] {name}", flush=True)


def _render(scene, cam, **kw):
    rast = raster.Rasterizer(cam, device=_dev(), **kw)
    fr = rast.render(*raster.scene_tensors(scene, _dev(), kw.get("feat_dtype", "f32")), want_last=True,
                     want_idx=True)
    torch.cuda.synchronize()
    return rast, fr


@pytest.mark.parametrize("K,tile", [(1, 8), (4, 8), (8, 16), (16, 8)])
def test_by_weight_small_against_oracle(K, tile):
    _case(f"by weight small K={K} tile={tile}")
    scene, cam = scenes.parity_small()
    rast, fr = _render(scene, cam, tile=tile, topk=K, topk_mode="weight")
    ref = oracle.render_scene(scene, cam, K=K, by_weight=True)
    check_image(fr, ref, rast, 0, scene.channels, K, f"by weight K={K}")
    # it differs from the first-K reading somewhere (the test would be vacuous otherwise)
    if K < 16:
        first = oracle.render_scene(scene, cam, K=K)
        assert not np.array_equal(first.idx[..., :K], ref.idx[..., :K])


def test_by_weight_workload_full_image():
    _case("by weight 300k")
    scene, cam = scenes.topk_scene()
    rast, fr = _render(scene, cam, tile=8, topk=8, topk_mode="weight")
    ref = oracle.render_scene(scene, cam, K=8, by_weight=True)
    check_image(fr, ref, rast, 0, scene.channels, 8, "by weight 300k")


def test_by_weight_with_k_above_every_count_is_the_full_blend():
    """K = 16 by weight keeps every contributor of a pixel with at most 16:
    there the weights, the order and the sums are those of the full blend,
    bit for bit."""
    _case("by weight vs full blend")
    scene, cam = scenes.parity_small()
    _, fw = _render(scene, cam, tile=8, topk=16, topk_mode="weight")
    _, ff = _render(scene, cam, tile=8, topk=0)
    few = (ff.n <= 16)
    assert int(few.sum()) > 0.9 * few.numel()
    assert torch.equal(fw.feat[few], ff.feat[few])
    assert torch.equal(fw.T, ff.T)


def test_by_weight_unsupported_combinations():
    _case("by weight unsupported")
    scene, cam = scenes.parity_small()
    tens = raster.scene_tensors(scene, _dev())
    rast = raster.Rasterizer(cam, device=_dev(), tile=8, topk=8, topk_mode="weight", schedule="grid")
    with pytest.raises(_lib.FastSegSimError):
        rast.render(*tens)
    rast = raster.Rasterizer(cam, device=_dev(), tile=8, topk=8, topk_mode="weight")
    fr = rast.render(*tens, want_last=True)
    g = torch.ones(cam.height * cam.width, scene.channels, device=_dev())
    with pytest.raises(_lib.FastSegSimError):
        rast.render_backward(*tens, fr, g)
    torch.cuda.synchronize()
