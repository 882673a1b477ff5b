"""Seeded synthetic scenes and cameras for the surfel feature rasterizer.

This module only draws inputs: surfel parameters (centre, two tangent scales,
rotation quaternion, opacity, per-surfel feature vector) and pinhole cameras.
It holds none of the rendering arithmetic, so both the GPU path and the CPU
oracle can take their inputs from here.

The surfel parameterisation follows the paper's preliminaries (Sec. 3.1,
Eq. 1): centre p, tangent scales (r_u, r_v), a tangent frame given here as a
unit quaternion (w, x, y, z), an opacity o in (0, 1) and a feature vector c of
C channels (16 semantic + 32 instance channels in the paper's experiments,
Sec. 4.1).  The paper's datasets (ScanNet-V2 / ScanNet++ scenes with trained
surfels) are not available; the generators below stand in for them with
clustered scenes of similar density.

Draw order inside each generator is fixed (means, scales, quaternions,
opacity, features) so that a seed fully determines a scene.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Scene:
    means: np.ndarray      # (N, 3) float32, world space
    scales: np.ndarray     # (N, 2) float32, linear tangent scales (r_u, r_v)
    quats: np.ndarray      # (N, 4) float32, (w, x, y, z), not necessarily unit
    opacity: np.ndarray    # (N,)   float32 in (0, 1)
    feats: np.ndarray      # (N, C) float32, row-major
    cluster: np.ndarray | None = None  # (N,) int32 cluster id, clustered scenes only
    centres: np.ndarray | None = None  # (n_clusters, 3) cluster centres

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def channels(self) -> int:
        return int(self.feats.shape[1])

    def subset(self, idx: np.ndarray) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.scales[idx].copy(), self.quats[idx].copy(),
                     self.opacity[idx].copy(), self.feats[idx].copy(),
                     None if self.cluster is None else self.cluster[idx].copy(), self.centres)

    def with_channels(self, feats: np.ndarray) -> "Scene":
        return Scene(self.means, self.scales, self.quats, self.opacity,
                     np.ascontiguousarray(feats, dtype=np.float32), self.cluster, self.centres)


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    R and t map world points to camera space: p_c = R p + t.  Pixel (px, py)
    covers [px, px+1) x [py, py+1); its sample point is the pixel centre.
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray = field(default_factory=lambda: np.eye(3, dtype=np.float32))
    t: np.ndarray = field(default_factory=lambda: np.zeros(3, dtype=np.float32))
    z_near: float = 0.2

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.ascontiguousarray(self.t, dtype=np.float32).reshape(3)
        # every scalar is representable in float32 so both sides read the same value
        self.fx = float(np.float32(self.fx))
        self.fy = float(np.float32(self.fy))
        self.cx = float(np.float32(self.cx))
        self.cy = float(np.float32(self.cy))
        self.z_near = float(np.float32(self.z_near))

    @property
    def pixels(self) -> int:
        return self.width * self.height


def centred_camera(width: int, height: int, focal: float | None = None) -> Camera:
    f = float(width if focal is None else focal)
    return Camera(width, height, f, f, width / 2.0, height / 2.0)


def _unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _normal32_into(rng: np.random.Generator, out: np.ndarray, scale: float, rows: int = 16384) -> None:
    """Fill a 2-D float32 array with N(0, scale^2) by the Box-Muller transform
    of float32 uniforms, chunk by chunk (few large temporaries)."""
    n, c = out.shape
    for r0 in range(0, n, rows):
        blk = out[r0:r0 + rows]
        size = blk.size
        half = (size + 1) // 2
        u1 = rng.random(half, dtype=np.float32)
        u2 = rng.random(half, dtype=np.float32)
        rad = np.sqrt(np.float32(-2.0) * np.log1p(-u1)) * np.float32(scale)
        ang = np.float32(2.0 * np.pi) * u2
        flat = blk.reshape(-1)
        flat[:half] = rad * np.cos(ang)
        flat[half:] = (rad * np.sin(ang))[:size - half]


def _log_uniform(rng: np.random.Generator, lo: float, hi: float, shape) -> np.ndarray:
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=shape)).astype(np.float32)


def _sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def uniform_scene(n: int, *, seed: int = 0, xy: float = 1.0, z: tuple[float, float] = (2.0, 6.0),
                  scale_range: tuple[float, float] = (0.005, 0.05), rgb: int = 3,
                  feat_channels: int = 16) -> Scene:
    """Uniform box scene: the parity workload with 2,000 surfels.

    means x, y ~ U[-xy, xy], z ~ U[z0, z1]; scales log-uniform; rotations uniform
    on SO(3); opacity = sigmoid(N(0, 1)); features = RGB ~ U(0, 1) followed by
    ``feat_channels`` channels ~ N(0, 1).
    """
    rng = np.random.default_rng(seed)
    means = np.empty((n, 3), np.float32)
    means[:, 0:2] = rng.uniform(-xy, xy, size=(n, 2))
    means[:, 2] = rng.uniform(z[0], z[1], size=n)
    scales = _log_uniform(rng, scale_range[0], scale_range[1], (n, 2))
    quats = _unit_quats(rng, n)
    opacity = _sigmoid(rng.standard_normal(n)).astype(np.float32)
    feats = np.concatenate([rng.uniform(0.0, 1.0, size=(n, rgb)),
                            rng.standard_normal((n, feat_channels))], axis=1).astype(np.float32)
    return Scene(means, scales, quats, opacity, np.ascontiguousarray(feats))


def clustered_scene(n: int, channels: int, *, seed: int = 0, box: tuple[float, float, float] = (10.0, 10.0, 4.0),
                    n_clusters: int = 50, sigma: float = 0.3,
                    scale_range: tuple[float, float] = (0.002, 0.03),
                    opacity_mu: float = 1.0, opacity_sd: float = 1.0) -> Scene:
    """Clustered scene standing in for a reconstructed indoor scene.

    Box a x b x c: x in [-a/2, a/2], y in [-b/2, b/2], z in [a, a + c] (the near
    face sits at z = a, so a focal length equal to the image width fills the
    width at the near face).  Cluster centres are uniform in the box; each
    surfel picks a cluster uniformly and is placed at centre + N(0, sigma^2 I).
    Features are a scaled one-hot code of the cluster id plus small noise:
    c_j = [j == cluster] * N(1, 0.1) + N(0, 0.05^2).
    """
    rng = np.random.default_rng(seed)
    a, b, c = box
    centres = np.stack([rng.uniform(-a / 2, a / 2, n_clusters),
                        rng.uniform(-b / 2, b / 2, n_clusters),
                        rng.uniform(a, a + c, n_clusters)], axis=1)
    cluster = rng.integers(0, n_clusters, size=n)
    means = (centres[cluster] + sigma * rng.standard_normal((n, 3))).astype(np.float32)
    scales = _log_uniform(rng, scale_range[0], scale_range[1], (n, 2))
    quats = _unit_quats(rng, n)
    opacity = _sigmoid(rng.normal(opacity_mu, opacity_sd, size=n)).astype(np.float32)
    feats = np.empty((n, channels), np.float32)
    _normal32_into(rng, feats, 0.05)
    hot = cluster % channels
    feats[np.arange(n), hot] += (1.0 + 0.1 * rng.standard_normal(n)).astype(np.float32)
    return Scene(means, scales, quats, opacity, feats, cluster.astype(np.int32), centres.astype(np.float32))


def lookat_camera(eye, target, width: int, height: int, down=(0.0, 1.0, 0.0), focal: float | None = None) -> Camera:
    """Camera at ``eye`` looking at ``target`` with image-down along ``down``."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    dn = np.asarray(down, np.float64)
    right = np.cross(dn, fwd)
    right /= np.linalg.norm(right)
    dn = np.cross(fwd, right)
    R = np.stack([right, dn, fwd], axis=0)          # rows: camera x, y, z axes in world
    t = -R @ eye
    f = float(width if focal is None else focal)
    return Camera(width, height, f, f, width / 2.0, height / 2.0, R.astype(np.float32), t.astype(np.float32))


RESOLUTIONS = ((320, 240), (640, 480), (960, 540), (1280, 720))


def random_lookat_views(n_views: int, *, seed: int = 0, centre=(0.0, 0.0, 22.5), dist=(25.0, 35.0),
                        max_angle_deg: float = 60.0, target_sd: float = 1.0,
                        resolutions=RESOLUTIONS) -> list[Camera]:
    """Uneven-resolution look-at views around a scene box (multi-view workload).

    eye = centre + d * dir with d ~ U[dist], dir uniform on the cap within
    ``max_angle_deg`` of -z; target = centre + N(0, target_sd^2 I); resolution
    drawn uniformly from ``resolutions``; focal length = image width.
    """
    rng = np.random.default_rng(seed)
    cams = []
    centre = np.asarray(centre, np.float64)
    cos_max = np.cos(np.deg2rad(max_angle_deg))
    for _ in range(n_views):
        d = rng.uniform(*dist)
        cz = rng.uniform(cos_max, 1.0)
        phi = rng.uniform(0.0, 2 * np.pi)
        sz = np.sqrt(max(0.0, 1.0 - cz * cz))
        direction = np.array([sz * np.cos(phi), sz * np.sin(phi), -cz])
        eye = centre + d * direction
        target = centre + target_sd * rng.standard_normal(3)
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        cams.append(lookat_camera(eye, target, w, h))
    return cams


# ---------------------------------------------------------------------------
# The workloads used by tests and the benchmark.
# ---------------------------------------------------------------------------

def needle_scene(n: int = 400, *, seed: int = 5) -> tuple[Scene, Camera]:
    """Long, very thin surfels at shallow slopes, 512x128: the footprint
    crosses pixel centres only every few tens of pixels, so many surfels touch
    a handful of tiles spread over more than 16 tile columns (the sparse
    footprints whose tiles the compact tile cache cannot hold)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.015, 0.04, n) * rng.choice([-1.0, 1.0], n)
    quats = np.stack([np.cos(th / 2), 0 * th, 0 * th, np.sin(th / 2)], 1).astype(np.float32)
    means = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n), np.full(n, 4.0)], 1).astype(np.float32)
    scales = np.stack([rng.uniform(0.3, 0.6, n), np.full(n, 2e-5)], 1).astype(np.float32)
    opacity = np.full(n, 0.9, np.float32)
    feats = rng.standard_normal((n, 4)).astype(np.float32)
    return Scene(means, scales, quats, opacity, feats), centred_camera(512, 128)


def border_scene(n: int = 3000, *, seed: int = 3) -> tuple[Scene, Camera]:
    """Surfels centred just outside (or just inside) the four edges of a
    160x96 view, by -0.5 to 1.5 times their approximate projected cutoff
    radius: many reach into the image with their centre outside it, many
    miss it by a little (the cases a view test before projection must get
    right)."""
    rng = np.random.default_rng(seed)
    cam = centred_camera(160, 96)
    z = rng.uniform(2.0, 6.0, n)
    s = np.exp(rng.uniform(np.log(0.01), np.log(0.08), n))
    rpx = np.sqrt(2.0 * np.log(0.9 * 255.0)) * s * cam.fx / z
    side = rng.integers(0, 4, n)
    t = rng.uniform(0.0, 1.0, n)
    off = rng.uniform(-0.5, 1.5, n) * rpx
    px = np.where(side == 0, -off, np.where(side == 1, cam.width + off, t * cam.width))
    py = np.where(side == 2, -off, np.where(side == 3, cam.height + off, t * cam.height))
    means = np.stack([(px - cam.cx) * z / cam.fx, (py - cam.cy) * z / cam.fy, z], 1).astype(np.float32)
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    scales = np.stack([s, s * rng.uniform(0.3, 1.0, n)], 1).astype(np.float32)
    feats = rng.standard_normal((n, 4)).astype(np.float32)
    return Scene(means, scales, q.astype(np.float32), np.full(n, 0.9, np.float32), feats), cam


def parity_small(seed: int = 0) -> tuple[Scene, Camera]:
    """2,000 surfels, 128x128, RGB + 16 feature channels (C = 19)."""
    return uniform_scene(2000, seed=seed), centred_camera(128, 128)


def topk_scene(seed: int = 0, n: int = 300_000, channels: int = 64) -> tuple[Scene, Camera]:
    """300k clustered surfels in a 10x10x4 box, 640x480, C = 64."""
    return clustered_scene(n, channels, seed=seed, box=(10.0, 10.0, 4.0)), centred_camera(640, 480)


def backward_scene(seed: int = 0, n: int = 200_000, channels: int = 128) -> tuple[Scene, Camera]:
    """200k clustered surfels, 640x480, C = 128 (gradient workload)."""
    return clustered_scene(n, channels, seed=seed, box=(10.0, 10.0, 4.0)), centred_camera(640, 480)


def large_scene(channels: int, seed: int = 0, n: int = 1_000_000) -> Scene:
    """1M clustered surfels in a 20x20x5 box (cluster sigma 0.3)."""
    return clustered_scene(n, channels, seed=seed, box=(20.0, 20.0, 5.0))


def headline(seed: int = 0, channels: int = 128) -> tuple[Scene, Camera]:
    """1M surfels, 1280x720 (fx = fy = 1280), C = 128: the throughput workload."""
    return large_scene(channels, seed=seed), centred_camera(1280, 720)


def multiview(seed: int = 0, n_views: int = 16, channels: int = 128) -> tuple[Scene, list[Camera]]:
    """1M surfels seen from 16 look-at views of uneven resolution."""
    return large_scene(channels, seed=seed), random_lookat_views(n_views, seed=seed + 1)


def upstream_grad(height: int, width: int, channels: int, seed: int = 1) -> np.ndarray:
    """Upstream gradient dL/dF ~ N(0, 1), layout (H, W, C)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((height, width, channels)).astype(np.float32)


def crop_near_cluster(scene: Scene, count: int, cluster: int = 0) -> np.ndarray:
    """Indices of the ``count`` surfels nearest to a cluster centre (sorted)."""
    assert scene.centres is not None
    d = np.linalg.norm(scene.means.astype(np.float64) - scene.centres[cluster].astype(np.float64), axis=1)
    return np.sort(np.argsort(d, kind="stable")[:count])


@dataclass
class Queries:
    feats: np.ndarray   # (Q, D) float32 query features
    means: np.ndarray   # (Q, 3) float32 query centres
    covs: np.ndarray    # (Q, 6) float32 covariances (xx, xy, xz, yy, yz, zz)


def instance_inputs(scene: Scene, num_queries: int = 32, dim: int = 32, *, seed: int = 0,
                    sigma: float = 0.6) -> tuple[np.ndarray, Queries]:
    """Instance features for every surfel and instance queries (the inputs of
    the query-guided instance labels, Sec. 3.3; the paper uses 32-dimensional
    features).  Query j sits at a cluster centre (or a random surfel of an
    unclustered scene) with a random covariance R diag(s^2) R^T, s in
    sigma * [0.5, 2]; its feature is a random unit vector times 3.  A surfel's
    feature is the feature of the query of its cluster (cluster id mod Q;
    nearest query centre for unclustered scenes) plus N(0, 0.5^2) noise."""
    rng = np.random.default_rng(seed + 7919)
    Q, n = num_queries, scene.n
    if scene.centres is not None and scene.cluster is not None:
        centres = scene.centres[np.arange(Q) % len(scene.centres)].astype(np.float64)
        owner = scene.cluster % Q
    else:
        centres = scene.means[rng.integers(0, n, Q)].astype(np.float64)
        d2 = ((scene.means[:, None, :].astype(np.float64) - centres[None]) ** 2).sum(-1)
        owner = np.argmin(d2, axis=1)
    covs = np.empty((Q, 6))
    for j in range(Q):
        a = rng.standard_normal((3, 3))
        R, _ = np.linalg.qr(a)
        s = sigma * rng.uniform(0.5, 2.0, 3)
        S = (R * s ** 2) @ R.T
        covs[j] = [S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]]
    qf = rng.standard_normal((Q, dim))
    qf = 3.0 * qf / np.linalg.norm(qf, axis=1, keepdims=True)
    feats = qf[owner] + 0.5 * rng.standard_normal((n, dim))
    return (np.ascontiguousarray(feats, np.float32),
            Queries(qf.astype(np.float32), centres.astype(np.float32), covs.astype(np.float32)))
