"""Independent textbook geometry used to pin the oracle (tests only).

Nothing here comes from the oracle: the rotation comes from scipy, the
ray-splat intersection is solved as a world-space ray-plane linear system,
and the blend is a pure-Python loop over the paper's Eq. (2).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation


def rotation(q_wxyz) -> np.ndarray:
    q = np.asarray(q_wxyz, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def ray_plane_uv(mean, scale, quat, cam, x, y):
    """Tangent coordinates (u, v) where the ray through pixel point (x, y)
    meets the surfel plane p + u r_u t_u + v r_v t_v (Sec. 3.1, Eq. 1)."""
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    Rinv = np.linalg.inv(R)   # float32 storage leaves R orthonormal only to ~1e-7
    centre = -Rinv @ t
    d_cam = np.array([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, 1.0])
    d_w = Rinv @ d_cam
    Rq = rotation(quat)
    tu, tv = Rq[:, 0], Rq[:, 1]
    A = np.stack([d_w, -scale[0] * tu, -scale[1] * tv], axis=1)
    lam, u, v = np.linalg.solve(A, np.asarray(mean, np.float64) - centre)
    return u, v, lam


def camera_depth(mean, cam) -> float:
    return float((np.asarray(cam.R, np.float64) @ np.asarray(mean, np.float64) + np.asarray(cam.t, np.float64))[2])


def brute_blend(scene, cam, pixels, *, K=0, by_weight=False, alpha_min=1 / 255, alpha_max=0.99, t_stop=1e-4):
    """Pure-Python front-to-back blend (Eq. 2; Top-K of Sec. 3.4 as the first K
    accepted surfels, or with by_weight the K contributors of the whole walk
    with the largest weights alpha T).  Every surfel is assumed to be in front
    of the camera.  Returns per pixel (F, T, order of contributors)."""
    out = []
    n = scene.means.shape[0]
    z = [np.float32(camera_depth(scene.means[i], cam)) for i in range(n)]
    order = sorted(range(n), key=lambda i: (z[i].view(np.uint32), i))
    for (px, py) in pixels:
        x, y = px + 0.5, py + 0.5
        F = np.zeros(scene.feats.shape[1])
        T = 1.0
        who = []
        walk = []   # (weight, position, surfel) of every contributor
        for i in order:
            u, v, _ = ray_plane_uv(scene.means[i], scene.scales[i].astype(np.float64), scene.quats[i], cam, x, y)
            o = float(scene.opacity[i])
            alpha = min(alpha_max, o * np.exp(-0.5 * (u * u + v * v)))
            if alpha < alpha_min:
                continue
            if T * (1 - alpha) < t_stop:
                break
            walk.append((alpha * T, len(walk), i))
            if not by_weight:
                F += alpha * T * scene.feats[i].astype(np.float64)
                who.append(i)
            T *= 1 - alpha
            if K and not by_weight and len(who) == K:
                break
        if by_weight:
            top = sorted(walk, key=lambda t: (-t[0], t[1]))[:K] if K else walk
            for w, _, i in sorted(top, key=lambda t: t[1]):
                F += w * scene.feats[i].astype(np.float64)
                who.append(i)
        out.append((F, T, who))
    return out
