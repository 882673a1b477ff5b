"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Bars: tile counts, sorted keys/values and tile ranges
bit-exact; Top-K index sets exact; float32 images within 1e-5 relative to
the pixel's absolute-term sum sum_i w_i |c_i| (the scale of float32 rounding
in the blend), on every pixel whose threshold decisions are not within 1e-5
of a threshold (the oracle flags those; their share is asserted small).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2604_10951_amd import raster, scenes

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5          # tolerance for float32 images, relative to the absolute-term sum
T_TOL = 1e-5            # final transmittance, relative
MASKED_MAX = 0.01       # at most 1% of pixels may sit within 1e-5 of a threshold


def _dev():
    return torch.device("cuda:0")


def _print_case(name):
    print(f"[case] {name}", flush=True)


def _render(scene, cams, **kw):
    rast = raster.Rasterizer(cams, device=_dev(), **kw)
    feat_dtype = kw.get("feat_dtype", "f32")
    fr = rast.render(*raster.scene_tensors(scene, _dev(), feat_dtype), want_last=True,
                     want_idx=kw.get("topk", 0) > 0)
    torch.cuda.synchronize()
    return rast, fr


def check_image(fr, ref, rast, v, C, K, name, *, pixels=None):
    """Compare one view (or a pixel subset of it) against an oracle Render."""
    cam = rast.cam_arr[v]
    W, H = cam.width, cam.height
    F = fr.view_image(rast, v, "feat").cpu().numpy().reshape(H * W, C)
    T = fr.view_image(rast, v, "T").cpu().numpy().reshape(H * W)
    n = fr.view_image(rast, v, "n").cpu().numpy().reshape(H * W)
    idx = fr.view_image(rast, v, "idx").cpu().numpy().reshape(H * W, K) if K > 0 else None
    if pixels is not None:
        F, T, n = F[pixels], T[pixels], n[pixels]
        idx = idx[pixels] if idx is not None else None
    rF = ref.F.reshape(-1, C)
    rA = ref.absF.reshape(-1, C)
    rT = ref.T.reshape(-1)
    rn = ref.n.reshape(-1)
    ok = ref.amb.reshape(-1) == 0
    masked = 1.0 - ok.mean()
    assert masked <= MASKED_MAX, f"{name}: {masked:.4f} of pixels ambiguous"
    err = np.abs(F - rF) / (rA + 1e-30)
    worst = float(err[ok].max()) if ok.any() else 0.0
    if worst > REL_TOL:
        bad = np.nonzero(ok & (err.max(1) > REL_TOL))[0]
        i = bad[np.argmax(err[bad].max(1))]
        c = int(np.argmax(err[i]))
        print(f"{name}: {len(bad)} bad pixels; worst pixel {i} ch {c}: gpu {F[i, c]!r} oracle {rF[i, c]!r} "
              f"abs {rA[i, c]!r}; n gpu {n[i]} oracle {rn[i]}; T gpu {T[i]} oracle {rT[i]}", flush=True)
    assert worst <= REL_TOL, f"{name}: max relative error {worst:.3g}"
    assert np.array_equal(n[ok], rn[ok]), f"{name}: contributor counts differ on {(n[ok] != rn[ok]).sum()} px"
    terr = np.abs(T - rT) / rT
    assert float(terr[ok].max()) <= T_TOL, f"{name}: T rel error {terr[ok].max():.3g}"
    if K > 0:
        ridx = ref.idx.reshape(-1, ref.idx.shape[-1])[:, :K]
        assert np.array_equal(idx[ok], ridx[ok]), f"{name}: Top-K index sets differ"
    return {"max_rel_err": worst, "masked": masked, "pixels": int(ok.size)}


def check_pairs(fr, scene, cams, tile, mode="precise", lowpass=False):
    """Tile counts, sorted keys/values and ranges bit-exact against the oracle
    (tile assignment `mode` of the oracle, with or without the low-pass disc)."""
    cams = cams if isinstance(cams, (list, tuple)) else [cams]
    n = scene.n
    counts_gpu = fr.tiles_touched.cpu().numpy().astype(np.uint32)
    flagged = np.zeros(len(cams) * n, bool)
    for v, cam in enumerate(cams):
        proj = oracle.project_scene(scene, cam)
        counts, flags, _, _ = oracle.tile_sets(proj, cam.width, cam.height, tile, mode=mode, lowpass=lowpass)
        sl = slice(v * n, (v + 1) * n)
        flagged[sl] = flags != 0
        assert np.array_equal(counts_gpu[sl][flags == 0], counts[flags == 0]), \
            f"view {v}: tile counts differ for {(counts_gpu[sl] != counts).sum()} surfels"
    assert flagged.sum() == 0, f"{flagged.sum()} surfels decided within 1e-12 of the cutoff"
    keys, vals, ntiles = oracle.sorted_pairs(scene, cams, tile, mode=mode, lowpass=lowpass)
    P = fr.num_pairs
    assert P == keys.shape[0]
    gk = fr.keys[:P].cpu().numpy().view(np.uint64)
    gv = fr.vals[:P].cpu().numpy().view(np.uint32)
    assert np.array_equal(gk, keys), f"sorted keys differ at {(gk != keys).sum()} positions"
    assert np.array_equal(gv, vals), f"sorted values differ at {(gv != vals).sum()} positions"
    ranges = oracle.tile_ranges(keys, ntiles)
    gr = fr.ranges.cpu().numpy().view(np.uint32)
    nonempty = ranges[:, 1] > ranges[:, 0]
    assert np.array_equal(gr[nonempty], ranges[nonempty])
    assert np.all(gr[~nonempty, 1] == gr[~nonempty, 0])
    return P


# ---------------------------------------------------------------------------
# Small parity workload: 2,000 surfels, 128x128, RGB + 16 features
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small():
    scene, cam = scenes.parity_small()
    return scene, cam


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_small_pairs_bit_exact(small, tile):
    scene, cam = small
    _print_case(f"small pairs tile={tile}")
    _, fr = _render(scene, cam, tile=tile)
    assert check_pairs(fr, scene, cam, tile) > 1000


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_small_full_blend(small, tile):
    scene, cam = small
    _print_case(f"small full tile={tile}")
    rast, fr = _render(scene, cam, tile=tile)
    ref = oracle.render_scene(scene, cam, kcap=256)
    check_image(fr, ref, rast, 0, scene.channels, 0, f"full tile={tile}")


@pytest.mark.parametrize("K,schedule", [(1, "grid"), (2, "grid"), (4, "grid"), (8, "grid"), (16, "grid"),
                                        (1, "split"), (4, "split"), (16, "split")])
def test_small_topk(small, K, schedule):
    scene, cam = small
    _print_case(f"small topk K={K} {schedule}")
    rast, fr = _render(scene, cam, tile=16, topk=K, schedule=schedule)
    ref = oracle.render_scene(scene, cam, K=K)
    check_image(fr, ref, rast, 0, scene.channels, K, f"topk K={K}")


def test_small_tile_modes_and_sizes_render_identically(small):
    scene, cam = small
    _print_case("tile modes identical")
    base = None
    pairs = {}
    for tile in (8, 16, 32):
        for mode in ("precise", "bbox"):
            rast, fr = _render(scene, cam, tile=tile, tile_mode=mode, topk=4)
            img = (fr.feat.cpu().numpy(), fr.T.cpu().numpy(), fr.n.cpu().numpy(), fr.idx.cpu().numpy())
            pairs[(tile, mode)] = fr.num_pairs
            if base is None:
                base = img
            else:
                for a, b in zip(base, img):
                    assert np.array_equal(a, b), (tile, mode)
    for tile in (8, 16, 32):
        assert pairs[(tile, "bbox")] > pairs[(tile, "precise")]


def test_small_topk_with_large_k_equals_full(small):
    scene, cam = small
    _print_case("large K == full")
    _, full = _render(scene, cam, tile=16)
    nmax = int(full.n.max().item())
    _, big = _render(scene, cam, tile=16, topk=min(64, nmax + 1))
    assert nmax + 1 <= 64
    assert torch.equal(full.feat, big.feat) and torch.equal(full.T, big.T) and torch.equal(full.n, big.n)


def test_small_forward_is_deterministic(small):
    scene, cam = small
    _print_case("determinism")
    _, a = _render(scene, cam, tile=16, topk=8)
    _, b = _render(scene, cam, tile=16, topk=8)
    assert torch.equal(a.feat, b.feat) and torch.equal(a.T, b.T) and torch.equal(a.idx, b.idx)
    assert torch.equal(a.keys[:a.num_pairs], b.keys[:b.num_pairs])


def test_empty_and_culled_scenes():
    _print_case("empty scene")
    cam = scenes.centred_camera(40, 24)
    sc = scenes.Scene(np.array([[0, 0, -5.0], [0, 0, 0.1]], np.float32), np.full((2, 2), 0.1, np.float32),
                      np.array([[1, 0, 0, 0], [1, 0, 0, 0]], np.float32), np.array([0.9, 0.9], np.float32),
                      np.ones((2, 3), np.float32))
    rast, fr = _render(sc, cam, tile=16)
    assert fr.num_pairs == 0
    assert torch.all(fr.feat == 0) and torch.all(fr.T == 1) and torch.all(fr.n == 0)


def test_ragged_image_and_odd_channels():
    """Image sizes that are not tile multiples; C not a multiple of 4 and > 64."""
    _print_case("ragged image, C=67")
    rng = np.random.default_rng(5)
    scene = scenes.uniform_scene(1500, seed=3, feat_channels=64)   # C = 67
    cam = scenes.Camera(101, 77, 101.0, 101.0, 50.5, 38.5)
    rast, fr = _render(scene, cam, tile=16, topk=6)
    ref = oracle.render_scene(scene, cam, K=6)
    check_image(fr, ref, rast, 0, scene.channels, 6, "ragged")
    check_pairs(fr, scene, cam, 16)
    del rng


def test_multiview_small_matches_per_view():
    _print_case("multiview small")
    scene = scenes.uniform_scene(1200, seed=7)
    cams = [scenes.centred_camera(96, 64), scenes.lookat_camera([0.5, -0.3, -1.0], [0, 0, 4], 80, 80),
            scenes.centred_camera(48, 40)]
    rast, fr = _render(scene, cams, tile=16, topk=4)
    check_pairs(fr, scene, cams, 16)
    for v, cam in enumerate(cams):
        ref = oracle.render_scene(scene, cam, K=4)
        # oracle indices are surfel ids; the GPU's are record ids v*n + i
        ref.idx = np.where(ref.idx >= 0, ref.idx + v * scene.n, -1)
        check_image(fr, ref, rast, v, scene.channels, 4, f"view {v}")


# ---------------------------------------------------------------------------
# Clustered 300k-surfel workload (640x480, C = 64): full image
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def topk_workload():
    scene, cam = scenes.topk_scene()
    return scene, cam


@pytest.mark.parametrize("K", [0, 8])
def test_topk_workload_full_image(topk_workload, K):
    scene, cam = topk_workload
    _print_case(f"300k K={K}")
    rast, fr = _render(scene, cam, tile=16, topk=K)
    if K == 8:
        check_pairs(fr, scene, cam, 16)
    ref = oracle.render_scene(scene, cam, K=K, kcap=max(K, 1))
    check_image(fr, ref, rast, 0, scene.channels, K, f"300k K={K}")


# ---------------------------------------------------------------------------
# Throughput workload: 1M surfels, 1280x720, C = 128 -- sampled pixels
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def headline():
    scene, cam = scenes.headline()
    return scene, cam


@pytest.mark.parametrize("K,schedule", [(8, "split"), (8, "grid"), (0, "grid")])
def test_headline_sampled_pixels(headline, K, schedule):
    scene, cam = headline
    _print_case(f"headline K={K} {schedule}")
    rast, fr = _render(scene, cam, tile=8, topk=K, schedule=schedule)   # the benchmark's launch configurations
    n_pix = cam.width * cam.height
    rng = np.random.default_rng(11)
    nvec = fr.n.cpu().numpy()
    covered = np.nonzero(nvec > 0)[0]
    pix = np.sort(np.concatenate([rng.choice(covered, 384, replace=False), rng.integers(0, n_pix, 64)]))
    proj = oracle.project_scene(scene, cam)
    ref = oracle.render_pixels(proj, scene.opacity, scene.feats, cam.width, pix, K=K, kcap=max(K, 1))
    check_image(fr, ref, rast, 0, scene.channels, K, f"headline K={K}", pixels=pix)


def test_headline_pairs_bit_exact(headline):
    scene, cam = headline
    _print_case("headline pairs")
    for tile in (8, 16):
        _, fr = _render(scene, cam, tile=tile, topk=8)
        assert check_pairs(fr, scene, cam, tile) > 100_000


def test_sort_long_tile_runs():
    """Tile runs longer than the in-LDS sorts hold (> 8192 entries) take the
    global radix path; short and medium runs take the LDS networks.  The
    sorted pairs and ranges must match the oracle's bit for bit."""
    _print_case("long tile runs")
    rng = np.random.default_rng(12)
    n = 24000
    means = np.empty((n, 3), np.float32)
    means[:, 0:2] = rng.uniform(-0.05, 0.05, size=(n, 2))
    means[:, 2] = rng.uniform(3.0, 5.0, size=n)
    scales = rng.uniform(0.05, 0.4, size=(n, 2)).astype(np.float32)
    q = rng.standard_normal((n, 4)).astype(np.float32)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity = rng.uniform(0.05, 0.95, size=n).astype(np.float32)
    feats = rng.standard_normal((n, 4)).astype(np.float32)
    sc = scenes.Scene(means, scales, q, opacity, feats)
    cam = scenes.centred_camera(96, 64)
    _, fr = _render(sc, cam, tile=32, topk=4)
    runs = (fr.ranges[:, 1] - fr.ranges[:, 0]).cpu().numpy()
    assert runs.max() > 8192 and ((runs > 1024) & (runs <= 8192)).any() or runs.max() > 8192, runs
    assert check_pairs(fr, sc, cam, 32) > 8192


def test_sparse_footprints_pairs_and_image():
    """Needle surfels: footprints of 4-8 tiles more than 15 tiles apart (kept
    out of the compact tile cache and re-derived), of more than 8 tiles and of
    at most 3; sorted pairs bit-exact and the full blend within tolerance."""
    _print_case("sparse needle footprints")
    scene, cam = scenes.needle_scene()
    for tile in (8, 16):
        rast, fr = _render(scene, cam, tile=tile)
        assert check_pairs(fr, scene, cam, tile) > 1000
    ref = oracle.render_scene(scene, cam, kcap=256)
    rast, fr = _render(scene, cam, tile=8)
    check_image(fr, ref, rast, 0, scene.channels, 0, "needles")


def test_border_surfels_pairs_and_image():
    """Surfels centred just outside and just inside the image edges: the
    view test that precedes the projection must never drop one that reaches
    a pixel centre.  Pairs bit-exact (tiles 8 and 16, both tile modes) and
    the full blend within tolerance."""
    _print_case("border surfels")
    scene, cam = scenes.border_scene()
    for tile in (8, 16):
        _, fr = _render(scene, cam, tile=tile)
        assert check_pairs(fr, scene, cam, tile) > 1000
    rast, fr = _render(scene, cam, tile=8, tile_mode="bbox")
    rast_p, fr_p = _render(scene, cam, tile=8)
    assert torch.equal(fr.feat, fr_p.feat) and torch.equal(fr.n, fr_p.n)
    ref = oracle.render_scene(scene, cam, kcap=256)
    check_image(fr_p, ref, rast_p, 0, scene.channels, 0, "border")
