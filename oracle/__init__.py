"""CPU oracle for the Fast-SegSim surfel feature rasterizer (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links
or executes anything in this package, and this package shares no code with it.

Projection, tile sets, sorting, the blend and its gradient are plain C in
``fso.c`` (double precision, built with ``-ffp-contract=off``), called through
ctypes.  The linearised covariance analysis, the label read-out and the
query-guided instance labels are numpy in this file (double precision), as is
the finite-difference driver used to pin the analytic gradient.

Functions and the paper passage each follows:
  project        tangent frame, T, adj(T), cutoff, culling    Sec. 3.1 Eq. (1), Sec. 3.2 (T)
  tile_sets      per-pixel footprint test -> tiles            Sec. 3.2 (exact result of the
                                                               precise tile intersection; or the
                                                               linearised Sigma' ellipse, read
                                                               literally; optional low-pass disc)
  linearised_cov / linearised_tile_stats
                 the linearised projected covariance Sigma' and what tiles it misses
                                                               Sec. 3.2 (the printed formula, read literally)
  sort_pairs     (tile, depth) ordering                        Sec. 3.1 (depth-sorted surfels)
  render_image / render_pixels
                 front-to-back blend, full or Top-K            Sec. 3.1 Eq. (2), Sec. 3.4 F_TopK
  render_lists / render_tiled
                 the same blend walking each pixel's tile list  Sec. 3.1 Eq. (2) over the tile lists of
                                                               Sec. 3.2; depth and normal outputs
  normals        n = t_u x t_v in camera space, facing it     Sec. 3.1
  labels         per-pixel argmax channel of a render          Sec. 3.3, Sec. 3.5 (masks from blended
                                                               class / instance channels)
  query_density_ratio / instance_labels
                 per-Gaussian instance labels from queries    Sec. 3.3 (S, D, A, softmax)
  render_grad    chain rule of the blend (held decisions)     training through the renderer, Sec. 3.5
  finite_difference  central differences of render_image      (pins render_grad)

Parity status: every function is pinned by tests under ``tests/`` (closed
forms, brute force, invariants, finite differences).  The two readings the
paper leaves open -- the exact projective conic in place of the garbled
linearised covariance of Sec. 3.2, and "first K accepted contributors in depth
order" for the Top-K set of Sec. 3.4 -- are pinned by those invariants only;
the paper prints no worked values to pin them against.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfso.so")

# The thresholds are float32 numbers (the renderer's parameters are float32);
# the oracle uses their exact double values so both sides test the same bound.
ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = float(np.float32(0.99))
T_STOP = float(np.float32(1e-4))

_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u32 = ctypes.POINTER(ctypes.c_uint32)
_u64 = ctypes.POINTER(ctypes.c_uint64)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i8 = ctypes.POINTER(ctypes.c_int8)


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def load():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    I64, I32, D = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.fso_project.argtypes = [_d, _d, _d, _d, I64, _d, D, _i32, _u32, _d, _d, _d]
    lib.fso_surfel_d2_image.argtypes = [_d, I32, I32, _d]
    lib.fso_conic_bounds.argtypes = [_d, D, _d]
    lib.fso_conic_bounds.restype = I32
    lib.fso_tile_sets.argtypes = [_i32, _u32, _d, _d, _d, I64, I32, I32, I32, I32, I32, I32, I64, I64, _u32, _i8,
                                  _u64, _u32]
    lib.fso_tile_sets.restype = I64
    lib.fso_sort_pairs.argtypes = [_u64, _u32, I64]
    lib.fso_tile_ranges.argtypes = [_u64, I64, I64, _u32]
    lib.fso_render_pixels.argtypes = [_i32, _u32, _d, _d, _d, _d, _d, _d, I64, I32, I32, _i64, I64, I32, D, D, D,
                                      I32, I32, _d, _d, _d, _i32, _i32, _i32, _i32, _d]
    lib.fso_render_lists.argtypes = [_i32, _u32, _d, _d, _d, _d, _d, _d, I64, I32, I32, I32, I32, _u32, _u32, _i64,
                                     I64, I32, D, D, D, I32, I32, _d, _d, _d, _i32, _i32, _i32, _i32, _d]
    lib.fso_normals.argtypes = [_d, _d, I64, _d, _d]
    lib.fso_render_image.argtypes = [_i32, _u32, _d, _d, _d, _d, I64, I32, I32, I32, I32, D, D, D, I32, I32,
                                     _d, _d, _d, _i32, _i32, _i32, _i32]
    lib.fso_render_grad.argtypes = [_d, _d, _d, _d, _d, I64, I32, _d, I32, D, D, D, I32, _d, _d, _d, _d, _d, _d,
                                    _d, _d, _d, _d, _d]
    _lib = lib
    return lib


def camera_array(cam) -> np.ndarray:
    """Pack a camera (width, height, fx, fy, cx, cy, R, t, z_near) as 19 doubles."""
    return np.concatenate([[cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy],
                           np.asarray(cam.R, np.float64).reshape(9), np.asarray(cam.t, np.float64).reshape(3),
                           [cam.z_near]]).astype(np.float64)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Projection:
    valid: np.ndarray   # (N,) int32
    zkey: np.ndarray    # (N,) uint32, float32 bits of the centre depth
    T: np.ndarray       # (N, 3, 3) rows T1, T2, Tw
    H: np.ndarray       # (N, 3, 3) adj(T): h = H (x, y, 1)
    k2: np.ndarray      # (N,) cutoff 2 ln(o / alpha_min)


def project(means, scales, quats, opacity, cam, alpha_min: float = ALPHA_MIN) -> Projection:
    lib = load()
    means, scales, quats, opacity = _f64(means), _f64(scales), _f64(quats), _f64(opacity)
    n = means.shape[0]
    valid = np.zeros(n, np.int32)
    zkey = np.zeros(n, np.uint32)
    T = np.zeros((n, 3, 3))
    H = np.zeros((n, 3, 3))
    k2 = np.zeros(n)
    ca = camera_array(cam)
    lib.fso_project(_ptr(means, _d), _ptr(scales, _d), _ptr(quats, _d), _ptr(opacity, _d), n, _ptr(ca, _d),
                    float(alpha_min), _ptr(valid, _i32), _ptr(zkey, _u32), _ptr(T, _d), _ptr(H, _d), _ptr(k2, _d))
    return Projection(valid, zkey, T, H, k2)


def project_scene(scene, cam, alpha_min: float = ALPHA_MIN) -> Projection:
    return project(scene.means, scene.scales, scene.quats, scene.opacity, cam, alpha_min)


def surfel_d2_image(H: np.ndarray, width: int, height: int) -> np.ndarray:
    """u^2 + v^2 at every pixel centre for one projected surfel, (height, width)."""
    lib = load()
    H = _f64(H).reshape(9)
    out = np.zeros((height, width))
    lib.fso_surfel_d2_image(_ptr(H, _d), width, height, _ptr(out, _d))
    return out


def conic_bounds(H: np.ndarray, k2: float):
    lib = load()
    H = _f64(H).reshape(9)
    bb = np.zeros(4)
    ok = lib.fso_conic_bounds(_ptr(H, _d), float(k2), _ptr(bb, _d))
    return bb if ok else None


MODES = {"precise": 0, "linearised": 2}


def tile_sets(proj: Projection, width: int, height: int, tile: int, *, prefilter: bool = True,
              tile_offset: int = 0, val_offset: int = 0, pairs: bool = False, mode: str = "precise",
              lowpass: bool = False):
    """Per-surfel tile counts (and optionally the unsorted pair list).

    mode "precise": a tile holds a surfel iff one of its pixel centres is in
    the exact footprint u^2 + v^2 <= k^2; "linearised": iff one is in the
    linearised ellipse of Sec. 3.2; lowpass adds the low-pass disc
    2 |x - mu|^2 <= k^2.
    Returns (counts uint32 (N,), flags int8 (N,), keys uint64 (P,), vals uint32 (P,)).
    """
    lib = load()
    n = proj.valid.shape[0]
    counts = np.zeros(n, np.uint32)
    flags = np.zeros(n, np.int8)
    H = _f64(proj.H)
    T = _f64(proj.T)
    md = MODES[mode]
    total = lib.fso_tile_sets(_ptr(proj.valid, _i32), _ptr(proj.zkey, _u32), _ptr(T, _d), _ptr(H, _d),
                              _ptr(proj.k2, _d), n, width, height, tile, int(prefilter), md, int(lowpass),
                              tile_offset, val_offset, _ptr(counts, _u32), _ptr(flags, _i8), None, None)
    if total < 0:
        raise MemoryError("oracle tile_sets failed")
    keys = vals = None
    if pairs:
        keys = np.zeros(max(total, 1), np.uint64)
        vals = np.zeros(max(total, 1), np.uint32)
        lib.fso_tile_sets(_ptr(proj.valid, _i32), _ptr(proj.zkey, _u32), _ptr(T, _d), _ptr(H, _d),
                          _ptr(proj.k2, _d), n, width, height, tile, int(prefilter), md, int(lowpass), tile_offset,
                          val_offset, _ptr(counts, _u32), _ptr(flags, _i8), _ptr(keys, _u64), _ptr(vals, _u32))
        keys, vals = keys[:total], vals[:total]
    return counts, flags, keys, vals


def linearised_cov(T) -> tuple[np.ndarray, np.ndarray]:
    """Screen-space centre mu and covariance Sigma' = J J^T of one surfel from
    the local linearisation of Sec. 3.2 (its printed formula is garbled; read
    as the Jacobian of the projective map at the tangent origin):
    J[r, c] = (T[r, c] - mu_r T[w, c]) / T[w, 3] for r, c in {1, 2}, with
    mu_r = T[r, 3] / T[w, 3].  The surfel's tangent coordinates have unit
    variance (its scales are inside T)."""
    T = np.asarray(T, np.float64)
    mu = T[:2, 2] / T[2, 2]
    J = (T[:2, :2] - mu[:, None] * T[2, :2][None, :]) / T[2, 2]
    return mu, J @ J.T


def linearised_tile_stats(proj: Projection, width: int, height: int, tile: int) -> dict:
    """Tiles assigned by the linearised ellipse (x - mu)^T Sigma'^-1 (x - mu)
    <= k^2 (pixel centres inside it, as the exact assignment uses the exact
    footprint) against the exact per-pixel footprint d^2 <= k^2.  Counts:
    exact_pairs / lin_pairs (tile, surfel) pairs of each assignment; dropped =
    (surfel, pixel) contributions whose tile the linearised set lacks; extra =
    linearised tiles holding no exact pixel; affected = pixels losing at least
    one contribution; contributions = all exact (surfel, pixel) pairs."""
    ys, xs = np.mgrid[0:height, 0:width]
    cx, cy = xs + 0.5, ys + 0.5
    tile_of = (ys // tile) * ((width + tile - 1) // tile) + (xs // tile)
    out = {"exact_pairs": 0, "lin_pairs": 0, "dropped": 0, "extra": 0, "contributions": 0}
    affected = np.zeros((height, width), bool)
    for i in np.nonzero(proj.valid)[0]:
        ex = surfel_d2_image(proj.H[i], width, height) <= proj.k2[i]
        mu, S = linearised_cov(proj.T[i])
        P = np.linalg.inv(S)
        dx, dy = cx - mu[0], cy - mu[1]
        lin = P[0, 0] * dx * dx + 2.0 * P[0, 1] * dx * dy + P[1, 1] * dy * dy <= proj.k2[i]
        ex_t, lin_t = np.unique(tile_of[ex]), np.unique(tile_of[lin])
        out["exact_pairs"] += len(ex_t)
        out["lin_pairs"] += len(lin_t)
        out["extra"] += len(np.setdiff1d(lin_t, ex_t))
        drop = ex & ~np.isin(tile_of, lin_t)
        out["dropped"] += int(drop.sum())
        out["contributions"] += int(ex.sum())
        affected |= drop
    out["affected"] = int(affected.sum())
    return out


def sort_pairs(keys: np.ndarray, vals: np.ndarray):
    lib = load()
    keys = np.ascontiguousarray(keys, np.uint64).copy()
    vals = np.ascontiguousarray(vals, np.uint32).copy()
    lib.fso_sort_pairs(_ptr(keys, _u64), _ptr(vals, _u32), keys.shape[0])
    return keys, vals


def tile_ranges(keys: np.ndarray, num_tiles: int) -> np.ndarray:
    lib = load()
    keys = np.ascontiguousarray(keys, np.uint64)
    ranges = np.zeros((num_tiles, 2), np.uint32)
    if lib.fso_tile_ranges(_ptr(keys, _u64), keys.shape[0], num_tiles, _ptr(ranges, _u32)) != 0:
        raise ValueError("tile id out of range")
    return ranges


def sorted_pairs(scene, cams, tile: int, alpha_min: float = ALPHA_MIN, prefilter: bool = True,
                 mode: str = "precise", lowpass: bool = False):
    """Sorted (key, value) list over one or more views, tile ids offset per view
    in view order and values = view * N + surfel index."""
    cams = cams if isinstance(cams, (list, tuple)) else [cams]
    ks, vs, tile_off = [], [], 0
    n = scene.means.shape[0]
    for v, cam in enumerate(cams):
        proj = project_scene(scene, cam, alpha_min)
        _, _, k, val = tile_sets(proj, cam.width, cam.height, tile, prefilter=prefilter, tile_offset=tile_off,
                                 val_offset=v * n, pairs=True, mode=mode, lowpass=lowpass)
        ks.append(k)
        vs.append(val)
        tile_off += ((cam.width + tile - 1) // tile) * ((cam.height + tile - 1) // tile)
    keys, vals = sort_pairs(np.concatenate(ks), np.concatenate(vs))
    return keys, vals, tile_off


@dataclass
class Render:
    F: np.ndarray        # (..., C) blended features
    absF: np.ndarray     # (..., C) sum of w |c|: error scale of F
    T: np.ndarray        # (...)   final transmittance
    n: np.ndarray        # (...)   number of blended surfels
    idx: np.ndarray      # (..., kcap) blended surfel indices front to back, -1 padded
    amb: np.ndarray      # (...)   1 if a threshold decision lies within 1e-5 relative
    nclamp: np.ndarray   # (...)   how many contributors hit alpha_max
    D: np.ndarray | None = None      # (...)   blended depth sum_i w_i z_i(x) of the intersection points
    absD: np.ndarray | None = None   # (...)   sum_i w_i |z_i|
    N: np.ndarray | None = None      # (..., 3) blended camera-space normal sum_i w_i n_i
    absN: np.ndarray | None = None   # (..., 3) sum_i w_i |n_i|


def _with_geo(r: "Render", geo, shape):
    if geo is not None:
        g = geo.reshape(shape + (8,))
        r.D, r.absD, r.N, r.absN = g[..., 0], g[..., 1], g[..., 2:5], g[..., 5:8]
    return r


def normals(means, quats, cam) -> np.ndarray:
    """Camera-space unit normals n = R (t_u x t_v) of the surfels (Sec. 3.1),
    flipped to face the camera; (N, 3)."""
    lib = load()
    means, quats = _f64(means), _f64(quats)
    n = means.shape[0]
    out = np.zeros((n, 3))
    ca = camera_array(cam)
    lib.fso_normals(_ptr(means, _d), _ptr(quats, _d), n, _ptr(ca, _d), _ptr(out, _d))
    return out


def _render_common(proj, feats, opacity):
    return _f64(feats), _f64(opacity), _f64(proj.H)


def render_image(proj: Projection, opacity, feats, width: int, height: int, *, K: int = 0, kcap: int | None = None,
                 alpha_min: float = ALPHA_MIN, alpha_max: float = ALPHA_MAX, t_stop: float = T_STOP,
                 prefilter: bool = True, by_weight: bool = False) -> Render:
    """Whole-image render; with by_weight (K > 0) the K contributors of largest
    weight of the full walk are blended instead of the first K."""
    lib = load()
    feats, opacity, H = _render_common(proj, feats, opacity)
    n, C = feats.shape
    kcap = int(kcap if kcap is not None else (K if K > 0 else 64))
    npix = width * height
    F = np.zeros((npix, C))
    absF = np.zeros((npix, C))
    T = np.zeros(npix)
    nout = np.zeros(npix, np.int32)
    idx = np.zeros((npix, max(kcap, 1)), np.int32)
    amb = np.zeros(npix, np.int32)
    ncl = np.zeros(npix, np.int32)
    rc = lib.fso_render_image(_ptr(proj.valid, _i32), _ptr(proj.zkey, _u32), _ptr(H, _d), _ptr(proj.k2, _d),
                              _ptr(opacity, _d), _ptr(feats, _d), n, C, width, height, int(prefilter), alpha_min,
                              alpha_max, t_stop, -K if by_weight else K, kcap, _ptr(F, _d), _ptr(absF, _d), _ptr(T, _d),
                              _ptr(nout, _i32), _ptr(idx, _i32), _ptr(amb, _i32), _ptr(ncl, _i32))
    if rc != 0:
        raise MemoryError("oracle render_image failed")
    sh = (height, width)
    return Render(F.reshape(sh + (C,)), absF.reshape(sh + (C,)), T.reshape(sh), nout.reshape(sh),
                  idx.reshape(sh + (max(kcap, 1),))[..., :kcap], amb.reshape(sh), ncl.reshape(sh))


def render_pixels(proj: Projection, opacity, feats, width: int, pix, *, K: int = 0, kcap: int | None = None,
                  alpha_min: float = ALPHA_MIN, alpha_max: float = ALPHA_MAX, t_stop: float = T_STOP,
                  by_weight: bool = False, lowpass: bool = False, normals=None) -> Render:
    """Brute-force render of selected pixels (pix = py * width + px): every
    valid surfel is a candidate.  With normals ((N, 3) camera-space surfel
    normals) the depth and normal outputs are filled too."""
    lib = load()
    feats, opacity, H = _render_common(proj, feats, opacity)
    n, C = feats.shape
    pix = np.ascontiguousarray(pix, np.int64)
    m = pix.shape[0]
    kcap = int(kcap if kcap is not None else (K if K > 0 else 64))
    F = np.zeros((m, C))
    absF = np.zeros((m, C))
    T = np.zeros(m)
    nout = np.zeros(m, np.int32)
    idx = np.zeros((m, max(kcap, 1)), np.int32)
    amb = np.zeros(m, np.int32)
    ncl = np.zeros(m, np.int32)
    Tm = _f64(proj.T)
    nrm = None if normals is None else _f64(normals)
    geo = None if normals is None else np.zeros((m, 8))
    lib.fso_render_pixels(_ptr(proj.valid, _i32), _ptr(proj.zkey, _u32), _ptr(Tm, _d), _ptr(H, _d),
                          _ptr(proj.k2, _d), _ptr(opacity, _d), _ptr(feats, _d),
                          None if nrm is None else _ptr(nrm, _d), n, C, width, _ptr(pix, _i64), m, int(lowpass),
                          alpha_min, alpha_max, t_stop, -K if by_weight else K, kcap, _ptr(F, _d), _ptr(absF, _d),
                          _ptr(T, _d), _ptr(nout, _i32), _ptr(idx, _i32), _ptr(amb, _i32), _ptr(ncl, _i32),
                          None if geo is None else _ptr(geo, _d))
    return _with_geo(Render(F, absF, T, nout, idx[:, :kcap], amb, ncl), geo, (m,))


def render_lists(proj: Projection, opacity, feats, width: int, height: int, tile: int, vals, ranges, *, pix=None,
                 K: int = 0, kcap: int | None = None, alpha_min: float = ALPHA_MIN, alpha_max: float = ALPHA_MAX,
                 t_stop: float = T_STOP, by_weight: bool = False, lowpass: bool = False, normals=None) -> Render:
    """Render from sorted tile lists (one view, tile ids from 0, values =
    surfel indices): every pixel walks its tile's list front to back.  pix =
    None renders the whole image (outputs shaped (height, width, ...)),
    otherwise the listed pixels py * width + px."""
    lib = load()
    feats, opacity, H = _render_common(proj, feats, opacity)
    n, C = feats.shape
    kcap = int(kcap if kcap is not None else (K if K > 0 else 64))
    vals = np.ascontiguousarray(vals, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32).reshape(-1)
    pixa = None if pix is None else np.ascontiguousarray(pix, np.int64)
    m = width * height if pixa is None else pixa.shape[0]
    F = np.zeros((m, C))
    absF = np.zeros((m, C))
    T = np.zeros(m)
    nout = np.zeros(m, np.int32)
    idx = np.zeros((m, max(kcap, 1)), np.int32)
    amb = np.zeros(m, np.int32)
    ncl = np.zeros(m, np.int32)
    Tm = _f64(proj.T)
    nrm = None if normals is None else _f64(normals)
    geo = None if normals is None else np.zeros((m, 8))
    rc = lib.fso_render_lists(_ptr(proj.valid, _i32), _ptr(proj.zkey, _u32), _ptr(Tm, _d), _ptr(H, _d),
                              _ptr(proj.k2, _d), _ptr(opacity, _d), _ptr(feats, _d),
                              None if nrm is None else _ptr(nrm, _d), n, C, width, height, tile,
                              _ptr(vals, _u32), _ptr(ranges, _u32), None if pixa is None else _ptr(pixa, _i64), m,
                              int(lowpass), alpha_min, alpha_max, t_stop, -K if by_weight else K, kcap, _ptr(F, _d),
                              _ptr(absF, _d), _ptr(T, _d), _ptr(nout, _i32), _ptr(idx, _i32), _ptr(amb, _i32),
                              _ptr(ncl, _i32), None if geo is None else _ptr(geo, _d))
    if rc != 0:
        raise ValueError("render_lists: a list names an invalid surfel")
    sh = (height, width) if pixa is None else (m,)
    r = Render(F.reshape(sh + (C,)), absF.reshape(sh + (C,)), T.reshape(sh), nout.reshape(sh),
               idx.reshape(sh + (max(kcap, 1),))[..., :kcap], amb.reshape(sh), ncl.reshape(sh))
    return _with_geo(r, geo, sh)


def render_tiled(scene, cam, tile: int, *, mode: str = "precise", lowpass: bool = False, K: int = 0,
                 kcap: int | None = None, pix=None, geometry: bool = False, by_weight: bool = False,
                 alpha_min: float = ALPHA_MIN, alpha_max: float = ALPHA_MAX, t_stop: float = T_STOP) -> Render:
    """One view through the whole tiled definition: projection, tile sets of
    the given assignment mode (and low-pass option), sorted pairs, tile
    ranges, then render_lists (with depth and normal outputs if geometry)."""
    proj = project_scene(scene, cam, alpha_min)
    _, _, keys, vals = tile_sets(proj, cam.width, cam.height, tile, pairs=True, mode=mode, lowpass=lowpass)
    keys, vals = sort_pairs(keys, vals)
    ntiles = ((cam.width + tile - 1) // tile) * ((cam.height + tile - 1) // tile)
    ranges = tile_ranges(keys, ntiles)
    nrm = normals(scene.means, scene.quats, cam) if geometry else None
    return render_lists(proj, scene.opacity, scene.feats, cam.width, cam.height, tile, vals, ranges, pix=pix, K=K,
                        kcap=kcap, alpha_min=alpha_min, alpha_max=alpha_max, t_stop=t_stop, by_weight=by_weight,
                        lowpass=lowpass, normals=nrm)


def render_scene(scene, cam, *, K: int = 0, kcap: int | None = None, alpha_min: float = ALPHA_MIN,
                 alpha_max: float = ALPHA_MAX, t_stop: float = T_STOP, prefilter: bool = True,
                 feats=None, by_weight: bool = False) -> Render:
    proj = project_scene(scene, cam, alpha_min)
    return render_image(proj, scene.opacity, scene.feats if feats is None else feats, cam.width, cam.height, K=K,
                        kcap=kcap, alpha_min=alpha_min, alpha_max=alpha_max, t_stop=t_stop, prefilter=prefilter,
                        by_weight=by_weight)


def labels(r: Render, rel_tol: float = 0.0):
    """Segmentation label of every pixel of a render (Sec. 3.3, Sec. 3.5: the
    masks come from blending per-Gaussian class or instance scores as
    channels; the label is read as the best-scoring channel).

    Returns (label, score, near): label = the channel of largest F, the lowest
    one among equal maxima (0 for a pixel with no contributor); score = F at
    that channel; near = (..., C) mask of the channels that could still be
    the largest if every F[c] were off by up to rel_tol * absF[c] (a render in
    lower precision may pick any of them; near has one channel where the
    choice is certain)."""
    F, A = r.F, r.absF
    label = np.argmax(F, axis=-1)
    score = np.take_along_axis(F, label[..., None], axis=-1)[..., 0]
    lo = score - rel_tol * np.take_along_axis(A, label[..., None], axis=-1)[..., 0]
    near = F + rel_tol * A >= lo[..., None]
    return label, score, near


def _cov_matrix(c6) -> np.ndarray:
    xx, xy, xz, yy, yz, zz = (float(v) for v in c6)
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def query_density_ratio(points, query_mean, query_cov6) -> np.ndarray:
    """D(p_q, p_g) = phi(p_g) / phi(p_q) (Sec. 3.3), phi the density of the
    query's Gaussian N(p_q, Sigma_q), each evaluated in full (normalising
    constant included) and then divided."""
    S = _cov_matrix(query_cov6)
    P = np.linalg.inv(S)
    norm = 1.0 / np.sqrt((2.0 * np.pi) ** 3 * np.linalg.det(S))
    mu = _f64(query_mean).reshape(3)

    def phi(x):
        d = x - mu
        return norm * np.exp(-0.5 * np.einsum("ni,ij,nj->n", d, P, d))

    return phi(_f64(points).reshape(-1, 3)) / phi(mu[None])


def instance_labels(ins_feats, means, query_feats, query_means, query_covs) -> np.ndarray:
    """Instance label of every scene Gaussian (Sec. 3.3), in double precision:
    similarity S = sigmoid(f_q^T f_ins), proximity D = query_density_ratio,
    attention A = S D, label = softmax of A over the queries.  Returns
    (n, Q)."""
    f, fq = _f64(ins_feats), _f64(query_feats)
    S = 1.0 / (1.0 + np.exp(-(f @ fq.T)))
    D = np.stack([query_density_ratio(means, query_means[q], query_covs[q]) for q in range(fq.shape[0])], axis=1)
    E = np.exp(S * D)
    return E / E.sum(axis=1, keepdims=True)


@dataclass
class Grads:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    feats: np.ndarray
    abs: "Grads | None" = None   # absolute-term sums (error scale), if requested


def render_grad(means, scales, quats, opacity, feats, cam, g, *, K: int = 0, alpha_min: float = ALPHA_MIN,
                alpha_max: float = ALPHA_MAX, t_stop: float = T_STOP, prefilter: bool = True,
                with_abs: bool = False) -> Grads:
    """Gradient of sum(g * F) w.r.t. means, (activated) scales, raw quaternions,
    (activated) opacity and features; g has shape (H, W, C).  With with_abs,
    also the sums of absolute values of the terms of each gradient."""
    lib = load()
    means, scales, quats, opacity, feats = _f64(means), _f64(scales), _f64(quats), _f64(opacity), _f64(feats)
    n, C = feats.shape
    g = _f64(g).reshape(cam.height * cam.width, C)
    out = [np.zeros((n, 3)), np.zeros((n, 2)), np.zeros((n, 4)), np.zeros(n), np.zeros((n, C))]
    ab = [np.zeros((n, 3)), np.zeros((n, 2)), np.zeros((n, 4)), np.zeros(n), np.zeros((n, C))] if with_abs else None
    ca = camera_array(cam)
    aptr = [_ptr(a, _d) for a in ab] if with_abs else [None] * 5
    rc = lib.fso_render_grad(_ptr(means, _d), _ptr(scales, _d), _ptr(quats, _d), _ptr(opacity, _d), _ptr(feats, _d),
                             n, C, _ptr(ca, _d), int(prefilter), alpha_min, alpha_max, t_stop, K, _ptr(g, _d),
                             *[_ptr(a, _d) for a in out], *aptr)
    if rc != 0:
        raise MemoryError("oracle render_grad failed")
    return Grads(*out, abs=Grads(*ab) if with_abs else None)


# ---------------------------------------------------------------------------
# Finite differences on the pre-activation parameters
# ---------------------------------------------------------------------------

def _forward_loss(params, cam, g, K, alpha_min, alpha_max, t_stop, kcap):
    means, log_s, quats, logit_o, feats = params
    scales = np.exp(log_s)
    opacity = 1.0 / (1.0 + np.exp(-logit_o))
    proj = project(means, scales, quats, opacity, cam, alpha_min)
    r = render_image(proj, opacity, feats, cam.width, cam.height, K=K, kcap=kcap, alpha_min=alpha_min,
                     alpha_max=alpha_max, t_stop=t_stop)
    loss = float(np.sum(g * r.F))
    # signature of the discrete decisions a derivative cannot see: the depth
    # order of the surfels, which contributors hit the alpha clamp and, with
    # Top-K, the selected sets.  Surfels entering or leaving a footprint at
    # alpha = alpha_min change the loss by O(alpha_min) only.
    order = np.lexsort((np.arange(proj.zkey.shape[0]), proj.zkey))
    order = order[proj.valid[order] == 1]
    sig = [order, r.nclamp.copy()]
    if K > 0:
        sig += [r.n.copy(), r.idx.copy()]
    return loss, sig


def _same_sig(a, b) -> bool:
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def finite_difference(means, log_scales, quats, logit_opacity, feats, cam, g, coords, *, h: float = 1e-3,
                      K: int = 0, alpha_min: float = 1e-12, alpha_max: float = ALPHA_MAX, t_stop: float = 0.0,
                      kcap: int = 512):
    """Central differences of L = sum(g * F) for the listed scalar coordinates.

    coords: iterable of (group, index tuple) with group in
    {"means", "log_scales", "quats", "logit_opacity", "feats"}.  Returns a list
    of (value or None); None marks a coordinate whose discrete decisions
    (contributor lists, clamp states) differ between theta - h, theta and
    theta + h, where a central difference is not a derivative.
    """
    names = ["means", "log_scales", "quats", "logit_opacity", "feats"]
    base = [_f64(means).copy(), _f64(log_scales).copy(), _f64(quats).copy(), _f64(logit_opacity).copy(),
            _f64(feats).copy()]
    _, sig0 = _forward_loss(base, cam, g, K, alpha_min, alpha_max, t_stop, kcap)
    out = []
    for group, index in coords:
        gi = names.index(group)
        vals = []
        ok = True
        for sgn in (+1.0, -1.0):
            p = [a.copy() for a in base]
            p[gi][index] += sgn * h
            loss, sig = _forward_loss(p, cam, g, K, alpha_min, alpha_max, t_stop, kcap)
            ok = ok and _same_sig(sig, sig0)
            vals.append(loss)
        out.append((vals[0] - vals[1]) / (2 * h) if ok else None)
    return out
