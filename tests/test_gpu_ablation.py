"""The directions of the paper's Tab. 2 ablation (Sec. 4.3), on the
300k-surfel, 640x480 workload: the precise tile intersection lists fewer
(tile, surfel) pairs than the bounding-box assignment, Top-K walks fewer
list entries per tile than the full blend, and both together walk the
fewest.  Only the directions come from the paper (its scenes, resolution and
channel count differ); the counters are exact, so the test is deterministic."""
from __future__ import annotations

import json
import os

import pytest
import torch

from paper_2604_10951_amd import raster, scenes

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tab2_ablation.json")


def test_tab2_directions():
    print("[case] Tab. 2 directions 300k", flush=True)
    paper = json.load(open(GOLDEN))["rows"]
    scene, cam = scenes.topk_scene()
    dev = torch.device("cuda:0")
    tens = raster.scene_tensors(scene, dev)
    got = {}
    for name, mode, K in (("A_baseline", "bbox", 0), ("B_precise_tiles", "precise", 0), ("C_topk", "bbox", 8),
                          ("D_precise_tiles_topk", "precise", 8)):
        rast = raster.Rasterizer(cam, tile=8, topk=K, tile_mode=mode, device=dev)
        fr = rast.render(*tens)
        cnt = torch.zeros(4, dtype=torch.int64, device=dev)
        rast.render_nosync(*tens, rast.alloc_out(scene.channels), counters=cnt)
        torch.cuda.synchronize()
        got[name] = {"pairs": fr.num_pairs, "walked": int(cnt[0]), "blended": int(cnt[2])}
    print(got, flush=True)
    # A -> B: fewer listed pairs (paper: RN-Total 6.1e6 -> 3.9e6)
    assert paper["B_precise_tiles"]["rn_total"] < paper["A_baseline"]["rn_total"]
    assert got["B_precise_tiles"]["pairs"] < got["A_baseline"]["pairs"]
    assert got["D_precise_tiles_topk"]["pairs"] < got["C_topk"]["pairs"]
    # A -> C: Top-K processes fewer entries per tile (paper: RN/Tile 1230 -> 610)
    assert paper["C_topk"]["rn_per_tile"] < paper["A_baseline"]["rn_per_tile"]
    assert got["C_topk"]["walked"] < got["A_baseline"]["walked"]
    assert got["C_topk"]["blended"] < got["A_baseline"]["blended"]
    # D: both together walk the fewest entries
    assert paper["D_precise_tiles_topk"]["rn_per_tile"] == min(r["rn_per_tile"] for r in paper.values())
    assert got["D_precise_tiles_topk"]["walked"] == min(r["walked"] for r in got.values())
    # the tile mode never changes the image: blended pairs do not depend on it
    assert got["A_baseline"]["blended"] == got["B_precise_tiles"]["blended"]
    assert got["C_topk"]["blended"] == got["D_precise_tiles_topk"]["blended"]
