"""Pins of the oracle's paper-literal tile assignment (the linearised Sigma'
of Sec. 3.2), its tiled render, the 2D Gaussian splatting low-pass option and
the depth / normal outputs (Sec. 3.1) against what the mathematics fixes.

References: closed forms (a fronto-parallel surfel's screen Gaussian, a plane's
depth, its normal), the independent pure-Python blend of tests/_indep.py
(scipy rotation, world-space ray-plane solve, pinhole projection), the
linearised covariance pinned by finite differences in test_oracle_pins.py, and
the whole-image brute force the tiled render must reproduce exactly.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2604_10951_amd import scenes
from tests import _indep
from tests.test_oracle_pins import _fronto_scene, _tilted_scene


def _oblique_scene(n, seed):
    """Oblique surfels close to a rotated camera (strong perspective), 24x20:
    the linearised ellipse misses footprint pixels here."""
    rng = np.random.default_rng(seed)
    sc, cam = _tilted_scene(n, seed)
    # push them closer and make them larger: perspective distortion grows
    pc = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), rng.uniform(0.7, 1.4, n)], 1)
    Rd = cam.R.astype(np.float64)
    means = ((pc - cam.t.astype(np.float64)) @ Rd).astype(np.float32)
    scales = np.exp(rng.uniform(np.log(0.1), np.log(0.5), (n, 2))).astype(np.float32)
    return scenes.Scene(means, scales, sc.quats, sc.opacity, sc.feats), cam


def _ranges(keys, cam, tile):
    ntiles = ((cam.width + tile - 1) // tile) * ((cam.height + tile - 1) // tile)
    return oracle.tile_ranges(keys, ntiles)


# ---------------------------------------------------------------------------
# The tiled render: with the exact tile sets it is the brute-force blend
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tile,K", [(8, 0), (16, 4), (32, 1)])
def test_tiled_render_with_exact_tiles_equals_brute_force(tile, K):
    """Every footprint pixel's tile lists the surfel, so walking the tile
    lists blends exactly the brute-force candidates in the same order: the
    images are bit-identical (Eq. 2 / Top-K of Sec. 3.4)."""
    scene, cam = scenes.parity_small()
    tiled = oracle.render_tiled(scene, cam, tile, K=K)
    brute = oracle.render_scene(scene, cam, K=K)
    for f in ("F", "T", "n", "idx"):
        assert np.array_equal(getattr(tiled, f), getattr(brute, f)), f


def test_tiled_render_with_every_surfel_in_every_tile_equals_brute_force():
    """Lists holding every valid surfel (sorted by depth key, then index) in
    every tile: acceptance is per pixel, so the image is the brute force."""
    sc, cam = _tilted_scene(25, 4)
    proj = oracle.project_scene(sc, cam)
    tile = 8
    ntx, nty = (cam.width + tile - 1) // tile, (cam.height + tile - 1) // tile
    live = np.nonzero(proj.valid)[0]
    order = live[np.lexsort((live, proj.zkey[live]))].astype(np.uint32)
    vals = np.tile(order, ntx * nty)
    ranges = np.stack([np.arange(ntx * nty) * len(order), (np.arange(ntx * nty) + 1) * len(order)], 1)
    r = oracle.render_lists(proj, sc.opacity, sc.feats, cam.width, cam.height, tile, vals, ranges)
    b = oracle.render_image(proj, sc.opacity, sc.feats, cam.width, cam.height)
    assert np.array_equal(r.F, b.F) and np.array_equal(r.T, b.T) and np.array_equal(r.n, b.n)


# ---------------------------------------------------------------------------
# Linearised tile assignment (Sec. 3.2, read literally)
# ---------------------------------------------------------------------------

def _numpy_linearised_tiles(proj, i, cam, tile):
    """Tiles holding a pixel centre inside the linearised ellipse, from
    oracle.linearised_cov (whose J is pinned against central differences of
    the world-space projection) evaluated with numpy over every pixel."""
    mu, S = oracle.linearised_cov(proj.T[i])
    P = np.linalg.inv(S)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    dx, dy = xs + 0.5 - mu[0], ys + 0.5 - mu[1]
    q = P[0, 0] * dx * dx + 2 * P[0, 1] * dx * dy + P[1, 1] * dy * dy
    k2 = proj.k2[i]
    near = np.abs(q - k2) < 1e-9 * k2
    ntx = (cam.width + tile - 1) // tile
    tiles = np.unique((ys[q <= k2] // tile) * ntx + xs[q <= k2] // tile)
    return tiles, bool(near.any())


@pytest.mark.parametrize("seed,tile", [(7, 8), (8, 4 * 4), (21, 8)])
def test_linearised_tile_sets_equal_the_pinned_ellipse(seed, tile):
    sc, cam = _oblique_scene(30, seed)
    proj = oracle.project_scene(sc, cam)
    counts, flags, keys, vals = oracle.tile_sets(proj, cam.width, cam.height, tile, pairs=True, mode="linearised")
    assert flags.sum() == 0
    checked = 0
    for i in np.nonzero(proj.valid)[0]:
        ref, near = _numpy_linearised_tiles(proj, i, cam, tile)
        if near:
            continue
        got = np.sort((keys[vals == i] >> np.uint64(32)).astype(np.int64))
        assert np.array_equal(got, ref), i
        assert counts[i] == len(ref)
        checked += 1
    assert checked >= 10


def test_linearised_tiles_equal_exact_tiles_when_the_map_is_affine():
    """Fronto-parallel surfels, unrotated camera: the perspective map is affine
    on the tangent plane, so the linearised ellipse is the exact footprint."""
    sc, cam = _fronto_scene(40, 1)
    proj = oracle.project_scene(sc, cam)
    ce, fe, ke, ve = oracle.tile_sets(proj, cam.width, cam.height, 8, pairs=True)
    cl, fl, kl, vl = oracle.tile_sets(proj, cam.width, cam.height, 8, pairs=True, mode="linearised")
    assert fe.sum() == 0 and fl.sum() == 0 and ce.sum() > 0
    assert np.array_equal(ce, cl) and np.array_equal(ke, kl) and np.array_equal(ve, vl)


def test_linearised_lists_drop_exactly_the_missing_tiles():
    """The tiled render over the linearised lists equals the independent
    pure-Python blend restricted, per pixel, to the surfels whose pinned
    linearised ellipse reaches the pixel's tile; and on this scene it does
    differ from the exact image (contributions are dropped)."""
    sc, cam = _oblique_scene(30, 7)
    tile = 8
    proj = oracle.project_scene(sc, cam)
    ntx = (cam.width + tile - 1) // tile
    lin_tiles = {int(i): set(_numpy_linearised_tiles(proj, i, cam, tile)[0].tolist())
                 for i in np.nonzero(proj.valid)[0]}
    lin = oracle.render_tiled(sc, cam, tile, mode="linearised")
    exact = oracle.render_tiled(sc, cam, tile)
    differ = np.nonzero((lin.n != exact.n).reshape(-1))[0]
    assert len(differ) > 0, "scene should show dropped contributions"
    pixels = [(int(p % cam.width), int(p // cam.width)) for p in
              np.concatenate([differ[:12], np.arange(0, cam.width * cam.height, 37)])]
    ref = _indep.brute_blend(sc, cam, pixels,
                             allowed=lambda px, py, i: ((py // tile) * ntx + px // tile) in lin_tiles.get(i, ()))
    for (px, py), (F, T, who) in zip(pixels, ref):
        if lin.amb[py, px]:
            continue
        np.testing.assert_allclose(lin.F[py, px], F, rtol=1e-9, atol=1e-12)
        assert abs(lin.T[py, px] - T) <= 1e-9 * T
        assert lin.n[py, px] == len(who)


def test_linearised_tile_counts_agree_with_the_numpy_analysis():
    sc, cam = _oblique_scene(40, 9)
    proj = oracle.project_scene(sc, cam)
    st = oracle.linearised_tile_stats(proj, cam.width, cam.height, 8)
    cl, fl, _, _ = oracle.tile_sets(proj, cam.width, cam.height, 8, mode="linearised")
    assert fl.sum() == 0 and st["lin_pairs"] == int(cl.sum())


# ---------------------------------------------------------------------------
# The low-pass option (2D Gaussian splatting's screen-space filter)
# ---------------------------------------------------------------------------

def test_lowpass_subpixel_surfel_is_a_screen_gaussian():
    """A fronto-parallel surfel far smaller than a pixel: without the filter
    it covers no pixel centre; with it, each pixel gets alpha = o exp(-|x - mu|^2)
    (variance 1/2 px^2 around the pinhole image mu of the centre) wherever
    that beats the surfel's own response, which is everywhere here."""
    cam = scenes.Camera(16, 12, 20.0, 20.0, 8.3, 5.9)
    X, Y, Z = 0.011, -0.013, 2.0
    sc = scenes.Scene(np.array([[X, Y, Z]], np.float32), np.array([[0.004, 0.003]], np.float32),
                      np.array([[1, 0, 0, 0]], np.float32), np.array([0.8], np.float32),
                      np.array([[1.0, -2.0]], np.float32))
    plain = oracle.render_tiled(sc, cam, 8)
    assert plain.n.sum() == 0
    lp = oracle.render_tiled(sc, cam, 8, lowpass=True)
    mu = np.array([cam.fx * float(np.float32(X)) / float(np.float32(Z)) + cam.cx,
                   cam.fy * float(np.float32(Y)) / float(np.float32(Z)) + cam.cy])
    o = float(np.float32(0.8))
    sx, sy = float(np.float32(0.004)) * cam.fx / Z, float(np.float32(0.003)) * cam.fy / Z
    covered = 0
    for py in range(cam.height):
        for px in range(cam.width):
            dx, dy = px + 0.5 - mu[0], py + 0.5 - mu[1]
            d2 = min((dx / sx) ** 2 + (dy / sy) ** 2, 2 * (dx * dx + dy * dy))
            a = min(0.99, o * np.exp(-0.5 * d2))
            if a < oracle.ALPHA_MIN:
                assert lp.n[py, px] == 0
                continue
            covered += 1
            np.testing.assert_allclose(lp.F[py, px], a * np.array([1.0, -2.0]), rtol=1e-12)
    assert covered >= 4


def test_lowpass_changes_nothing_for_surfels_wider_than_the_filter():
    """Fronto-parallel surfels whose screen standard deviations exceed
    sqrt(1/2) px: u^2 + v^2 <= 2 |x - mu|^2 at every pixel, so the filter
    never wins and the images (and tile sets) are identical."""
    sc, cam = _fronto_scene(40, 2)
    # screen standard deviation f s / z >= 40 * 0.08 / 4 = 0.8 px in both axes
    scales = np.random.default_rng(2).uniform(0.08, 0.3, (sc.n, 2)).astype(np.float32)
    sc = scenes.Scene(sc.means, scales, sc.quats, sc.opacity, np.random.default_rng(3).standard_normal((sc.n, 3))
                      .astype(np.float32))
    assert np.all(sc.scales * cam.fx / sc.means[:, 2:3] >= 0.8)
    a = oracle.render_tiled(sc, cam, 8)
    b = oracle.render_tiled(sc, cam, 8, lowpass=True)
    assert np.array_equal(a.F, b.F) and np.array_equal(a.T, b.T) and np.array_equal(a.n, b.n)


@pytest.mark.parametrize("seed", [2, 5])
def test_lowpass_blend_and_tiles_match_pure_python(seed):
    """Tilted surfels with sub-pixel widths: the oracle's low-pass render (tiled
    route and per-pixel brute force) against the independent pure-Python
    blend, and the tiled route's tiles cover every pixel it blends."""
    sc, cam = _tilted_scene(30, seed)
    sc = scenes.Scene(sc.means, (sc.scales * 0.08).astype(np.float32), sc.quats, sc.opacity, sc.feats)
    tiled = oracle.render_tiled(sc, cam, 8, lowpass=True)
    plain = oracle.render_tiled(sc, cam, 8)
    assert tiled.n.sum() > plain.n.sum()        # the filter makes sub-pixel surfels visible
    proj = oracle.project_scene(sc, cam)
    pix = np.arange(cam.width * cam.height)
    brute = oracle.render_pixels(proj, sc.opacity, sc.feats, cam.width, pix, lowpass=True)
    ok = (tiled.amb.reshape(-1) == 0) & (brute.amb == 0)
    assert np.array_equal(tiled.n.reshape(-1)[ok], brute.n[ok])
    np.testing.assert_allclose(tiled.F.reshape(-1, 5)[ok], brute.F[ok], rtol=0, atol=0)
    pixels = [(px, py) for py in range(0, cam.height, 3) for px in range(0, cam.width, 2)]
    ref = _indep.brute_blend(sc, cam, pixels, lowpass=True)
    for (px, py), (F, T, who) in zip(pixels, ref):
        if tiled.amb[py, px]:
            continue
        np.testing.assert_allclose(tiled.F[py, px], F, rtol=1e-9, atol=1e-12)
        assert tiled.n[py, px] == len(who)


# ---------------------------------------------------------------------------
# Depth and normal outputs (Sec. 3.1)
# ---------------------------------------------------------------------------

def test_normals_face_the_camera_and_match_scipy():
    sc, cam = _tilted_scene(40, 3)
    nr = oracle.normals(sc.means, sc.quats, cam)
    for i in range(sc.n):
        ref = _indep.camera_normal(sc.quats[i], sc.means[i], cam)
        np.testing.assert_allclose(nr[i], ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(nr, axis=1), 1.0, rtol=1e-12)
    pc = sc.means.astype(np.float64) @ cam.R.astype(np.float64).T + cam.t.astype(np.float64)
    assert np.all(np.einsum("ij,ij->i", nr, pc) <= 0)


def test_depth_and_normal_of_a_fronto_parallel_surfel():
    """A surfel facing the camera at depth Z: every intersection point has
    depth Z and the normal is (0, 0, -1), so D = alpha Z and N = alpha (0, 0, -1)."""
    cam = scenes.Camera(20, 16, 24.0, 24.0, 10.2, 7.7)
    Z = 3.0
    sc = scenes.Scene(np.array([[0.05, -0.02, Z]], np.float32), np.array([[0.4, 0.3]], np.float32),
                      np.array([[1, 0, 0, 0]], np.float32), np.array([0.7], np.float32), np.ones((1, 1), np.float32))
    r = oracle.render_tiled(sc, cam, 8, geometry=True)
    alpha = 1.0 - r.T
    assert (r.n > 0).sum() > 20
    np.testing.assert_allclose(r.D, alpha * Z, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r.N[..., 2], -alpha, rtol=1e-12, atol=1e-15)
    assert np.all(r.N[..., :2] == 0)


@pytest.mark.parametrize("K", [0, 3])
def test_depth_and_normal_match_pure_python(K):
    """Tilted surfels: blended depth of the world-space ray-plane intersection
    points and blended scipy normals, against the oracle's tiled route."""
    sc, cam = _tilted_scene(30, 6)
    r = oracle.render_tiled(sc, cam, 8, K=K, geometry=True)
    pixels = [(px, py) for py in range(0, cam.height, 2) for px in range(0, cam.width, 3)]
    ref = _indep.brute_blend(sc, cam, pixels, K=K, geometry=True)
    n_cov = 0
    for (px, py), (F, T, who, D, N) in zip(pixels, ref):
        if r.amb[py, px]:
            continue
        n_cov += len(who) > 0
        np.testing.assert_allclose(r.D[py, px], D, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(r.N[py, px], N, rtol=1e-9, atol=1e-12)
    assert n_cov > 20


def test_depth_is_a_weighted_mean_of_contributor_depths():
    """D / (1 - T) lies between the nearest and farthest contributor's
    intersection depth; |N| <= 1 - T (a blend of unit vectors)."""
    scene, cam = scenes.parity_small()
    r = oracle.render_tiled(scene, cam, 16, geometry=True)
    cov = r.n > 0
    w = 1.0 - r.T[cov]
    mean_depth = r.D[cov] / w
    proj = oracle.project_scene(scene, cam)
    zc = proj.T[proj.valid == 1][:, 2, 2]
    assert mean_depth.min() > 0.5 * zc.min() and mean_depth.max() < 2.0 * zc.max()
    assert np.all(np.linalg.norm(r.N[cov], axis=-1) <= w * (1 + 1e-12))
    np.testing.assert_allclose(r.absD, np.abs(r.D), rtol=1e-12)   # every depth is positive
