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


def pinhole(point, cam):
    """Pixel coordinates of a world point through the camera (R, t, K)."""
    pc = np.asarray(cam.R, np.float64) @ np.asarray(point, np.float64) + np.asarray(cam.t, np.float64)
    return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])


def camera_normal(quat, mean, cam):
    """Camera-space unit normal R (t_u x t_v) of a surfel (Sec. 3.1), scaled to
    unit length (the float32 camera rotation is orthonormal only to ~1e-7) and
    flipped to face the camera."""
    Rq = rotation(quat)
    n = np.asarray(cam.R, np.float64) @ np.cross(Rq[:, 0], Rq[:, 1])
    n = n / np.linalg.norm(n)
    pc = np.asarray(cam.R, np.float64) @ np.asarray(mean, np.float64) + np.asarray(cam.t, np.float64)
    return -n if n @ pc > 0 else n


def brute_blend(scene, cam, pixels, *, K=0, by_weight=False, alpha_min=1 / 255, alpha_max=0.99, t_stop=1e-4,
                lowpass=False, allowed=None, geometry=False):
    """Pure-Python front-to-back blend (Eq. 2; Top-K of Sec. 3.4 as the first K
    accepted surfels, or with by_weight the K contributors of the whole walk
    with the largest weights alpha T).  Every surfel is assumed to be in front
    of the camera.  lowpass: response exp(-min(u^2 + v^2, 2 |x - mu|^2) / 2)
    with mu the pinhole image of the centre (the 2D Gaussian splatting filter).
    allowed(px, py, i): whether surfel i is on the pixel's list (default: all).
    Returns per pixel (F, T, order of contributors), plus (depth, normal) --
    the blended camera depth of the ray-plane intersection points and the
    blended camera-facing normals -- when geometry is set."""
    out = []
    n = scene.means.shape[0]
    z = [np.float32(camera_depth(scene.means[i], cam)) for i in range(n)]
    order = sorted(range(n), key=lambda i: (z[i].view(np.uint32), i))
    mus = [pinhole(scene.means[i], cam) for i in range(n)] if lowpass else None
    nrms = [camera_normal(scene.quats[i], scene.means[i], cam) for i in range(n)] if geometry else None
    for (px, py) in pixels:
        x, y = px + 0.5, py + 0.5
        F = np.zeros(scene.feats.shape[1])
        D, N = 0.0, np.zeros(3)
        T = 1.0
        who = []
        walk = []   # (weight, position, surfel, depth) of every contributor
        for i in order:
            if allowed is not None and not allowed(px, py, i):
                continue
            u, v, lam = ray_plane_uv(scene.means[i], scene.scales[i].astype(np.float64), scene.quats[i], cam, x, y)
            d2 = u * u + v * v
            if lowpass:
                d2 = min(d2, 2.0 * float(np.sum((np.array([x, y]) - mus[i]) ** 2)))
            o = float(scene.opacity[i])
            alpha = min(alpha_max, o * np.exp(-0.5 * d2))
            if alpha < alpha_min:
                continue
            if T * (1 - alpha) < t_stop:
                break
            walk.append((alpha * T, len(walk), i, lam))
            if not by_weight:
                F += alpha * T * scene.feats[i].astype(np.float64)
                if geometry:
                    D += alpha * T * lam
                    N += alpha * T * nrms[i]
                who.append(i)
            T *= 1 - alpha
            if K and not by_weight and len(who) == K:
                break
        if by_weight:
            top = sorted(walk, key=lambda t: (-t[0], t[1]))[:K] if K else walk
            for w, _, i, lam in sorted(top, key=lambda t: t[1]):
                F += w * scene.feats[i].astype(np.float64)
                if geometry:
                    D += w * lam
                    N += w * nrms[i]
                who.append(i)
        out.append((F, T, who, D, N) if geometry else (F, T, who))
    return out
