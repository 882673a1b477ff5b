"""Per-pixel segmentation labels (fs_render_labels, Sec. 3.3 and 3.5): the
argmax epilogue of the split Top-K render.

Two bars: against the argmax of the feature image fs_render_forward writes
from the same sorted lists (same kernels, same float32 sums: labels, scores,
transmittance and counts bit for bit), and against the oracle's labels on
every pixel whose label the float32 tolerance cannot flip."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2604_10951_amd import _lib, raster, scenes
from tests.test_gpu_parity import MASKED_MAX, REL_TOL

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


def _case(name):
    print(f"[case] {name}", flush=True)


def _bf16_round(feats: np.ndarray) -> np.ndarray:
    return torch.from_numpy(feats).to(torch.bfloat16).to(torch.float32).numpy()


def _both(scene, cams, **kw):
    """Feature render and label render of one rasterizer (one set of lists)."""
    rast = raster.Rasterizer(cams, device=_dev(), schedule="split", **kw)
    tens = raster.scene_tensors(scene, _dev(), kw.get("feat_dtype", "f32"))
    fr = rast.render(*tens)
    lab = rast.render_labels(tens[4])
    torch.cuda.synchronize()
    return rast, fr, lab


def _check_against_features(fr, lab, name):
    F = fr.feat.cpu().numpy()
    want = np.argmax(F, axis=1)                     # first maximum: the lowest channel on ties
    got = lab["label"].cpu().numpy()
    assert np.array_equal(got, want), f"{name}: {(got != want).sum()} labels differ from argmax(F)"
    score = lab["score"].cpu().numpy()
    assert np.array_equal(score, F[np.arange(F.shape[0]), want]), f"{name}: scores differ"
    assert np.array_equal(lab["T"].cpu().numpy(), fr.T.cpu().numpy()), f"{name}: T differs"
    assert np.array_equal(lab["n"].cpu().numpy(), fr.n.cpu().numpy()), f"{name}: counts differ"


def _check_against_oracle(rast, lab, ref, v, pixels, name):
    """GPU labels of view v (or of `pixels` of it) against oracle.labels."""
    cam = rast.cam_arr[v]
    sl = slice(cam.pixel_offset, cam.pixel_offset + cam.width * cam.height)
    got = lab["label"][sl].cpu().numpy()
    score = lab["score"][sl].cpu().numpy()
    if pixels is not None:
        got, score = got[pixels], score[pixels]
    C = ref.F.shape[-1]
    rF, rA = ref.F.reshape(-1, C), ref.absF.reshape(-1, C)
    want, _, near = oracle.labels(ref, REL_TOL)
    want, near = want.reshape(-1), near.reshape(-1, C)
    ok = ref.amb.reshape(-1) == 0
    assert 1.0 - ok.mean() <= MASKED_MAX, f"{name}: too many ambiguous pixels"
    rows = np.arange(got.shape[0])
    assert np.all((got >= 0) & (got < C)), f"{name}: label out of range"
    allowed = near[rows, got]
    assert np.all(allowed[ok]), f"{name}: {(~allowed[ok]).sum()} labels outside the oracle's near-maximum set"
    certain = ok & (near.sum(1) == 1)
    assert np.array_equal(got[certain], want[certain])
    err = np.abs(score - rF[rows, got]) / (rA[rows, got] + 1e-30)
    assert float(err[ok].max()) <= REL_TOL, f"{name}: score error {err[ok].max():.3g}"
    return certain.mean()


@pytest.mark.parametrize("dtype,channels,K,mode", [
    ("f32", 16, 8, "first"),      # C = 19: vectors do not fit, general gather
    ("f32", 61, 8, "first"),      # C = 64: staged gather, 16 threads per pixel
    ("f32", 125, 16, "first"),    # C = 128, K = 16
    ("bf16", 125, 8, "first"),    # bfloat16 rows, 8 channels per vector
    ("f32", 297, 4, "first"),     # C = 300: more vectors than lanes, general gather
    ("f32", 61, 8, "weight"),     # Top-K by weight
    ("f32", 5, 4, "first"),       # C = 8: 4 threads per pixel
    ("f32", 29, 8, "first"),      # C = 32: 8 threads per pixel
    ("f32", 253, 8, "first"),     # C = 256: 64 threads per pixel (the reduction crosses wave halves)
    ("bf16", 509, 16, "first"),   # C = 512 bfloat16: 64 threads per pixel, K = 16
])
def test_labels_small_against_features_and_oracle(dtype, channels, K, mode):
    _case(f"labels small {dtype} C={channels + 3} K={K} {mode}")
    scene, _ = scenes.parity_small()
    rng = np.random.default_rng(channels)
    feats = np.concatenate([scene.feats[:, :3], rng.standard_normal((scene.n, channels))], 1).astype(np.float32)
    scene = scene.with_channels(feats)
    cam = scenes.centred_camera(101, 77)   # ragged against 8x8 blocks
    rast, fr, lab = _both(scene, cam, tile=8, topk=K, topk_mode=mode, feat_dtype=dtype)
    _check_against_features(fr, lab, "small")
    ref_feats = _bf16_round(scene.feats) if dtype == "bf16" else scene.feats
    ref = oracle.render_scene(scene, cam, K=K, feats=ref_feats, by_weight=mode == "weight")
    frac = _check_against_oracle(rast, lab, ref, 0, None, "small")
    assert frac > 0.3   # the comparison is not vacuous (empty pixels are ambiguous by construction)


@pytest.mark.parametrize("K,lowpass", [(24, False), (8, True)])
def test_labels_gather_forms(K, lowpass):
    """K above the selection's LDS lists (the general gather), and the
    low-pass response."""
    _case(f"labels gather form K={K} lowpass={lowpass}")
    scene, _ = scenes.parity_small()
    cam = scenes.centred_camera(101, 77)
    rast, fr, lab = _both(scene, cam, tile=8, topk=K, lowpass=lowpass)
    _check_against_features(fr, lab, f"K={K} lowpass={lowpass}")
    ref = oracle.render_tiled(scene, cam, 8, lowpass=lowpass, K=K, kcap=K)
    assert _check_against_oracle(rast, lab, ref, 0, None, f"K={K} lowpass={lowpass}") > 0.3


@pytest.mark.parametrize("mode", ["first", "weight"])
def test_label_counters_match_features(mode):
    """The counters (entries walked, rows, blended pairs, blocks) of a label
    render equal those of the feature render of the same lists."""
    _case(f"label counters {mode}")
    scene, cam = scenes.topk_scene()
    rast = raster.Rasterizer(cam, device=_dev(), tile=8, topk=8, topk_mode=mode, schedule="split")
    tens = raster.scene_tensors(scene, _dev())
    rast.render(*tens)
    c_feat = torch.zeros(4, dtype=torch.int64, device=_dev())
    c_lab = torch.zeros(4, dtype=torch.int64, device=_dev())
    rast.render_forward(tens[4], counters=c_feat)
    rast.render_labels(tens[4], counters=c_lab)
    torch.cuda.synchronize()
    assert torch.equal(c_feat, c_lab), (c_feat.tolist(), c_lab.tolist())
    assert int(c_lab[2]) > 0


def test_labels_two_views_and_empty_pixels():
    _case("labels two views")
    scene, _ = scenes.parity_small()
    cams = [scenes.centred_camera(128, 128), scenes.centred_camera(60, 44)]
    rast, fr, lab = _both(scene, cams, tile=16, topk=8)
    _check_against_features(fr, lab, "two views")
    for v, cam in enumerate(cams):
        ref = oracle.render_scene(scene, cam, K=8)
        _check_against_oracle(rast, lab, ref, v, None, f"view {v}")
    n = lab["n"].cpu().numpy()
    assert (n == 0).any()
    assert np.all(lab["label"].cpu().numpy()[n == 0] == 0) and np.all(lab["score"].cpu().numpy()[n == 0] == 0)


def test_labels_topk_workload():
    _case("labels 300k")
    scene, cam = scenes.topk_scene()
    rast, fr, lab = _both(scene, cam, tile=8, topk=8)
    _check_against_features(fr, lab, "300k")
    ref = oracle.render_scene(scene, cam, K=8)
    _check_against_oracle(rast, lab, ref, 0, None, "300k")


def test_labels_headline_workload():
    """1M surfels, 1280x720, C = 128, K = 8 (the benchmark's label frame):
    the whole image against argmax(F), sampled pixels against the oracle."""
    _case("labels headline")
    scene, cam = scenes.headline()
    rast, fr, lab = _both(scene, cam, tile=8, topk=8)
    _check_against_features(fr, lab, "headline")
    rng = np.random.default_rng(12)
    covered = np.nonzero(fr.n.cpu().numpy() > 0)[0]
    pix = np.sort(np.concatenate([rng.choice(covered, 384, replace=False),
                                  rng.integers(0, cam.width * cam.height, 64)]))
    proj = oracle.project_scene(scene, cam)
    ref = oracle.render_pixels(proj, scene.opacity, scene.feats, cam.width, pix, K=8)
    _check_against_oracle(rast, lab, ref, 0, pix, "headline")


def test_labels_without_score_and_argument_errors():
    _case("labels errors")
    scene, cam = scenes.parity_small()
    rast = raster.Rasterizer(cam, device=_dev(), tile=8, topk=8, schedule="split")
    tens = raster.scene_tensors(scene, _dev())
    rast.render(*tens)
    full = rast.render_labels(tens[4])
    bare = rast.render_labels(tens[4], want_score=False)
    assert bare["score"] is None
    assert torch.equal(full["label"], bare["label"])
    grid = raster.Rasterizer(cam, device=_dev(), tile=8, topk=8, schedule="grid")
    grid.render(*tens)
    with pytest.raises(_lib.FastSegSimError):
        grid.render_labels(tens[4])
    torch.cuda.synchronize()
