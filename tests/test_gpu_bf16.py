"""BF16 feature storage with float32 accumulation.

Against the FP64 oracle run on the bfloat16-rounded features the only error
left is float32 accumulation, so the image bar is the same 1e-5 relative to
the absolute-term sum.  Against the oracle on the original float32 features
the error is bounded by bfloat16 rounding (8 significant bits, so round to
nearest even has relative error at most 2^-8 per feature value) plus float32
accumulation: 2^-8 + 1e-5.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2604_10951_amd import raster, scenes
from tests.test_gpu_parity import check_image

pytestmark = pytest.mark.gpu

BF16_BOUND = 2.0 ** -8 + 1e-5


def _dev():
    return torch.device("cuda:0")


def _bf16_round(feats: np.ndarray) -> np.ndarray:
    return torch.from_numpy(feats).to(torch.bfloat16).to(torch.float32).numpy()


def _stats(fr, ref, rast, C, pixels=None):
    cam = rast.cam_arr[0]
    F = fr.view_image(rast, 0, "feat").cpu().numpy().reshape(-1, C)
    if pixels is not None:
        F = F[pixels]
    ok = ref.amb.reshape(-1) == 0
    e = (np.abs(F - ref.F.reshape(-1, C)) / (ref.absF.reshape(-1, C) + 1e-30))[ok]
    return float(e.max()), float(e.mean())


@pytest.mark.parametrize("channels,K", [(16, 0), (61, 4), (125, 8)])
def test_small_bf16(channels, K):
    print(f"[case] bf16 small C={channels + 3} K={K}", flush=True)
    scene = scenes.uniform_scene(2000, seed=4, feat_channels=channels)
    cam = scenes.centred_camera(128, 128)
    C = scene.channels
    rast = raster.Rasterizer(cam, tile=8, topk=K, feat_dtype="bf16", device=_dev())
    fr = rast.render(*raster.scene_tensors(scene, _dev(), "bf16"), want_idx=K > 0)
    torch.cuda.synchronize()
    rounded = _bf16_round(scene.feats)
    ref_b = oracle.render_scene(scene, cam, K=K, kcap=max(K, 1), feats=rounded)
    check_image(fr, ref_b, rast, 0, C, K, f"bf16 C={C} vs oracle(bf16 features)")
    ref_f = oracle.render_scene(scene, cam, K=K, kcap=max(K, 1))
    mx, mean = _stats(fr, ref_f, rast, C)
    print(f"bf16 C={C} K={K} vs oracle(f32 features): max {mx:.3g} mean {mean:.3g}", flush=True)
    assert mx <= BF16_BOUND


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_precision_workload_sampled(dtype):
    """1M surfels, 1280x720, C = 256 (two channel chunks), K = 16."""
    print(f"[case] C=256 K=16 {dtype}", flush=True)
    scene = scenes.large_scene(256)
    cam = scenes.centred_camera(1280, 720)
    rast = raster.Rasterizer(cam, tile=8, topk=16, feat_dtype=dtype, device=_dev())
    fr = rast.render(*raster.scene_tensors(scene, _dev(), dtype), want_idx=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    nvec = fr.n.cpu().numpy()
    pix = np.sort(np.concatenate([rng.choice(np.nonzero(nvec > 0)[0], 192, replace=False),
                                  rng.integers(0, cam.width * cam.height, 32)]))
    proj = oracle.project_scene(scene, cam)
    feats = _bf16_round(scene.feats) if dtype == "bf16" else scene.feats
    ref = oracle.render_pixels(proj, scene.opacity, feats, cam.width, pix, K=16)
    check_image(fr, ref, rast, 0, 256, 16, f"C=256 {dtype}", pixels=pix)
    # error of each output against the FP64 oracle on the float32 features
    ref_f = ref if dtype == "f32" else oracle.render_pixels(proj, scene.opacity, scene.feats, cam.width, pix, K=16)
    mx, mean = _stats(fr, ref_f, rast, 256, pixels=pix)
    Tg = fr.view_image(rast, 0, "T").cpu().numpy().reshape(-1)[pix]
    eT = np.abs(Tg.astype(np.float64) - ref_f.T.reshape(-1))
    print(f"{dtype} C=256 K=16 vs oracle(f32 features): features max {mx:.3g} mean {mean:.3g} (relative to "
          f"sum w|c|); T max {eT.max():.3g} mean {eT.mean():.3g} (absolute)", flush=True)
    if dtype == "bf16":
        assert mx <= BF16_BOUND
