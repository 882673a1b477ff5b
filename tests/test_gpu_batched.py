"""Batched multi-view form: persistent longest-first render, hipGraph-captured
frames, and the autotuner.  Scheduling changes only which workgroup renders a
block, so every image must be bit-identical to the one-workgroup-per-block
launch and to rendering the views one at a time."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2604_10951_amd import autotune, raster, scenes
from tests.test_gpu_parity import check_image, check_pairs

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


def _case(name):
    print(f"[case] {name}", flush=True)


def _views_small():
    scene = scenes.uniform_scene(1500, seed=9, feat_channels=61)          # C = 64
    cams = [scenes.centred_camera(96, 64), scenes.lookat_camera([0.4, -0.2, -1.0], [0, 0, 4], 80, 72),
            scenes.centred_camera(48, 40), scenes.lookat_camera([-0.6, 0.3, -0.5], [0.1, 0, 4], 64, 64)]
    return scene, cams


def _frame(rast, tens, **kw):
    fr = rast.render(*tens, **kw)
    torch.cuda.synchronize()
    return fr


@pytest.mark.parametrize("tile,batch", [(8, 16), (8, 32), (16, 16), (32, 32)])
def test_persistent_schedule_is_bit_identical(tile, batch):
    _case(f"persistent tile={tile} batch={batch}")
    scene, cams = _views_small()
    tens = raster.scene_tensors(scene, _dev())
    a = _frame(raster.Rasterizer(cams, tile=tile, batch=batch, topk=5, schedule="grid", device=_dev()), tens,
               want_idx=True)
    b = _frame(raster.Rasterizer(cams, tile=tile, batch=batch, topk=5, schedule="persistent", device=_dev()), tens,
               want_idx=True)
    for name in ("feat", "T", "n", "idx"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name


def test_batched_views_equal_single_views_and_oracle():
    _case("batched == per view")
    scene, cams = _views_small()
    tens = raster.scene_tensors(scene, _dev())
    rast = raster.Rasterizer(cams, tile=8, topk=6, schedule="persistent", device=_dev())
    fr = _frame(rast, tens, want_idx=True)
    check_pairs(fr, scene, cams, 8)
    for v, cam in enumerate(cams):
        single = raster.Rasterizer(cam, tile=8, topk=6, device=_dev())
        fs = _frame(single, tens, want_idx=True)
        assert torch.equal(fr.view_image(rast, v, "feat").reshape(-1, scene.channels), fs.feat)
        idx_b = fr.view_image(rast, v, "idx").reshape(-1, 6)
        assert torch.equal(torch.where(idx_b >= 0, idx_b - v * scene.n, idx_b), fs.idx)
        ref = oracle.render_scene(scene, cam, K=6)
        ref.idx = np.where(ref.idx >= 0, ref.idx + v * scene.n, -1)
        check_image(fr, ref, rast, v, scene.channels, 6, f"view {v}")


@pytest.mark.parametrize("schedule", ["persistent", "split"])
def test_graph_replay_matches_eager_and_follows_camera_updates(schedule):
    _case(f"graph replay ({schedule})")
    scene, cams = _views_small()
    tens = raster.scene_tensors(scene, _dev())
    rast = raster.Rasterizer(cams, tile=8, topk=4, schedule=schedule, device=_dev())
    graph = raster.FrameGraph(rast, tens)
    eager = raster.Rasterizer(cams, tile=8, topk=4, device=_dev())
    ref = _frame(eager, tens)
    for i in range(3):
        out = graph.replay()
        torch.cuda.synchronize()
        assert graph.pairs_fit()
        assert torch.equal(out["feat"], ref.feat) and torch.equal(out["T"], ref.T), i
        # unrelated eager work between replays
        _ = (tens[4] * 2).sum().item()
        _frame(eager, tens)
    moved = [scenes.lookat_camera([0.3 * k, -0.1, -1.2], [0, 0, 4], c.width, c.height) for k, c in enumerate(cams)]
    rast.set_cameras(moved)
    out = graph.replay()
    torch.cuda.synchronize()
    assert graph.pairs_fit()
    ref2 = _frame(raster.Rasterizer(moved, tile=8, topk=4, device=_dev()), tens)
    assert torch.equal(out["feat"], ref2.feat) and torch.equal(out["n"], ref2.n)


def test_sixteen_uneven_views_sampled_parity():
    """1M-surfel scene, 16 look-at views of uneven resolution, K = 8, one
    persistent batched frame; sampled pixels of every view against the oracle."""
    _case("16 views, 1M surfels")
    scene, cams = scenes.multiview()
    tens = raster.scene_tensors(scene, _dev())
    rast = raster.Rasterizer(cams, tile=8, topk=8, schedule="persistent", device=_dev())
    fr = _frame(rast, tens, want_idx=True)
    rng = np.random.default_rng(2)
    for v, cam in enumerate(cams):
        nvec = fr.view_image(rast, v, "n").reshape(-1).cpu().numpy()
        covered = np.nonzero(nvec > 0)[0]
        k = min(24, len(covered))
        pix = np.sort(np.concatenate([rng.choice(covered, k, replace=False),
                                      rng.integers(0, cam.width * cam.height, 8)]))
        proj = oracle.project_scene(scene, cam)
        ref = oracle.render_pixels(proj, scene.opacity, scene.feats, cam.width, pix, K=8)
        ref.idx = np.where(ref.idx >= 0, ref.idx + v * scene.n, -1)
        check_image(fr, ref, rast, v, scene.channels, 8, f"view {v} ({cam.width}x{cam.height})", pixels=pix)


def test_sixteen_views_split_schedule_as_benchmarked():
    """The batched frame exactly as the benchmark times it: the 1M-surfel
    scene, 16 uneven look-at views, 8x8 tiles, split Top-K render, K = 8.
    The frame has more tiles than the sort's LDS histogram holds, so the
    pairs go through the per-pair global count and scatter path: every
    sorted key, value and tile range is compared bit for bit with the
    oracle's, and sampled pixels of every view with the oracle's blend."""
    _case("16 views, split schedule, pairs + pixels")
    scene, cams = scenes.multiview()
    tens = raster.scene_tensors(scene, _dev())
    rast = raster.Rasterizer(cams, tile=8, topk=8, schedule="split", device=_dev())
    assert rast.total_tiles > 16384
    fr = _frame(rast, tens, want_idx=True)
    P = check_pairs(fr, scene, cams, 8)
    print(f"16 views: {rast.total_tiles} tiles, {P} pairs bit-exact", flush=True)
    rng = np.random.default_rng(4)
    for v, cam in enumerate(cams):
        nvec = fr.view_image(rast, v, "n").reshape(-1).cpu().numpy()
        covered = np.nonzero(nvec > 0)[0]
        k = min(32, len(covered))
        pix = np.unique(np.concatenate([rng.choice(covered, k, replace=False),
                                        rng.integers(0, cam.width * cam.height, 8)]))
        proj = oracle.project_scene(scene, cam)
        ref = oracle.render_pixels(proj, scene.opacity, scene.feats, cam.width, pix, K=8)
        ref.idx = np.where(ref.idx >= 0, ref.idx + v * scene.n, -1)
        check_image(fr, ref, rast, v, scene.channels, 8, f"split view {v} ({cam.width}x{cam.height})", pixels=pix)


def test_autotuner_picks_a_valid_config(tmp_path, monkeypatch):
    _case("autotune")
    monkeypatch.setenv("FASTSEGSIM_CACHE", str(tmp_path))
    scene, cams = _views_small()
    tens = raster.scene_tensors(scene, _dev())
    best = autotune.tune(cams, tens, topk=4, steps=2)
    assert best["tile"] in (8, 16, 32) and best["batch"] in (16, 32) and best["schedule"] in ("grid", "persistent", "split")
    assert len(best["trials"]) == 3 * 2 * 2 + 3 and best["ms"] == min(t["ms"] for t in best["trials"])
    again = autotune.tune(cams, tens, topk=4, steps=2)
    assert again["cached"] and again["tile"] == best["tile"]
