"""Host-side logic that needs no GPU: the benchmark's one-GPU guard, the
instance-input generator and the binding's argument checks."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_2604_10951_amd import raster, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def test_instance_inputs_are_seeded_and_well_formed():
    scene, _ = scenes.parity_small()
    f1, q1 = scenes.instance_inputs(scene, 7, 12, seed=3)
    f2, q2 = scenes.instance_inputs(scene, 7, 12, seed=3)
    assert f1.shape == (scene.n, 12) and f1.dtype == np.float32 and f1.flags.c_contiguous
    assert q1.feats.shape == (7, 12) and q1.means.shape == (7, 3) and q1.covs.shape == (7, 6)
    assert np.array_equal(f1, f2) and np.array_equal(q1.covs, q2.covs)
    for c in q1.covs.astype(np.float64):
        S = np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])
        assert np.all(np.linalg.eigvalsh(S) > 0)
    # clustered scenes put the queries on cluster centres
    big = scenes.clustered_scene(2000, 4, seed=1)
    _, qc = scenes.instance_inputs(big, 5, 8)
    np.testing.assert_array_equal(qc.means, big.centres[:5].astype(np.float32))


def test_instance_labels_binding_rejects_bad_tensors():
    good = torch.zeros((10, 32))
    with pytest.raises(ValueError):   # wrong feature dimension of the queries
        raster.instance_labels(good, torch.zeros((10, 3)), torch.zeros((4, 16)), torch.zeros((4, 3)),
                               torch.zeros((4, 6)))
    with pytest.raises(ValueError):   # float64 means
        raster.instance_labels(good, torch.zeros((10, 3), dtype=torch.float64), torch.zeros((4, 32)),
                               torch.zeros((4, 3)), torch.zeros((4, 6)))
    with pytest.raises(ValueError):   # host tensors never reach the library
        raster.instance_labels(good, torch.zeros((10, 3)), torch.zeros((4, 32)), torch.zeros((4, 3)),
                               torch.zeros((4, 6)))
