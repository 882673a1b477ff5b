"""Query-guided instance labels (fs_instance_labels, Sec. 3.3) against the
oracle, and the instance-label pipeline: per-Gaussian labels blended by the
split Top-K render and reduced to a per-pixel instance id.

Tolerance, from the float32 arithmetic: the dot product f_q . f_g of D
terms is off by at most D 2^-24 sum_d |f_q,d f_g,d|, which sigmoid (slope
<= 1/4) passes on to A scaled by 1/4; the proximity factor, the exponentials
and the reciprocal add a few ulp of A (in [0, 1]).  A softmax output moves by
at most twice the largest error of its row's A, relatively; 2^-18 covers the
rounding terms."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2604_10951_amd import raster, scenes
from tests.test_gpu_parity import REL_TOL

pytestmark = pytest.mark.gpu


def _dev():
    return torch.device("cuda:0")


def _case(name):
    print(f"[case] {name}", flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(_dev())


def _run(feats, means, q):
    out = raster.instance_labels(_t(feats), _t(means), _t(q.feats), _t(q.means), _t(q.covs))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _row_tol(feats, qfeats):
    D = feats.shape[1]
    absdot = np.abs(feats.astype(np.float64)) @ np.abs(qfeats.astype(np.float64)).T
    return 2.0 * (0.25 * D * 2.0 ** -24 * absdot.max(axis=1)) + 2.0 ** -18


def _check(got, feats, means, q, name):
    ref = oracle.instance_labels(feats, means, q.feats, q.means, q.covs)
    assert np.all(np.isfinite(got)), f"{name}: non-finite labels"
    tol = _row_tol(feats, q.feats)[:, None]
    err = np.abs(got - ref) / ref
    assert np.all(err <= tol), f"{name}: worst relative error {err.max():.3g} (bound {tol.max():.3g})"
    np.testing.assert_allclose(got.sum(1), 1.0, atol=got.shape[1] * 2.0 ** -22)
    return float(err.max())


@pytest.mark.parametrize("n,Q,D", [(1000, 1, 32), (1000, 5, 32), (1000, 8, 4), (1777, 32, 32), (300, 64, 36),
                                   (257, 13, 16),
                                   (1, 32, 32),     # matrix-core form, one live lane of 64
                                   (63, 32, 32),    # matrix-core form, a partial wave
                                   (500, 32, 48)])  # Q = 32 with another dimension: the vector form
def test_instance_labels_small(n, Q, D):
    _case(f"instance labels n={n} Q={Q} D={D}")
    scene = scenes.uniform_scene(n, seed=Q + D)
    feats, q = scenes.instance_inputs(scene, Q, D, seed=n)
    _check(_run(feats, scene.means, q), feats, scene.means, q, f"n={n} Q={Q} D={D}")


def test_instance_labels_workload_sampled():
    """1M Gaussians, 32 queries of dimension 32 (the bench's instance-label
    launch): 4096 sampled rows against the oracle (rows are independent), and
    every row finite and summing to 1."""
    _case("instance labels 1M")
    scene = scenes.large_scene(3)
    feats, q = scenes.instance_inputs(scene, 32, 32)
    got = _run(feats, scene.means, q)
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got.sum(1), 1.0, atol=32 * 2.0 ** -22)
    rows = np.sort(np.random.default_rng(4).choice(scene.n, 4096, replace=False))
    rows = np.concatenate([rows, [0, scene.n - 1]])
    _check(got[rows], feats[rows], scene.means[rows], q, "1M sampled")


def test_instance_pipeline_labels_against_oracle():
    """Instance labels -> split Top-K label render (C = Q channels) -> per-pixel
    instance id, against the oracle's chain (oracle instance labels, oracle
    blend, argmax)."""
    _case("instance pipeline")
    scene, cam = scenes.parity_small()
    Q = 8
    feats, q = scenes.instance_inputs(scene, Q, 32)
    lab = raster.instance_labels(_t(feats), _t(scene.means), _t(q.feats), _t(q.means), _t(q.covs))
    rast = raster.Rasterizer(cam, device=_dev(), tile=8, topk=8, schedule="split")
    tens = raster.scene_tensors(scene, _dev())
    rast.render(*tens[:4], lab)
    out = rast.render_labels(lab)
    torch.cuda.synchronize()
    ref_l = oracle.instance_labels(feats, scene.means, q.feats, q.means, q.covs)
    ref = oracle.render_scene(scene, cam, K=8, feats=ref_l)
    want, _, near = oracle.labels(ref, REL_TOL + float(_row_tol(feats, q.feats).max()))
    got = out["label"].cpu().numpy().reshape(cam.height, cam.width)
    ok = (ref.amb == 0) & (ref.n > 0)
    hit = np.take_along_axis(near, got[..., None].astype(np.int64), axis=-1)[..., 0]
    assert np.all(hit[ok]), f"{(~hit[ok]).sum()} pixel ids outside the oracle's near-maximum set"
    certain = ok & (near.sum(-1) == 1)
    assert certain.mean() > 0.3 and np.array_equal(got[certain], want[certain])
    assert len(np.unique(got[ok])) > 1   # more than one instance is visible
