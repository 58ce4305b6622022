"""The seeded generator: determinism and the structure of each workload recipe."""
import hashlib

import numpy as np
import torch

from paper_2302_09247_amd import synth


def _digest(w):
    h = hashlib.sha256()
    for t in (w.points, w.offsets, w.roi, w.lab):
        h.update(t.cpu().numpy().tobytes())
    return h.hexdigest()


def test_tiny64_recipe_and_determinism():
    a = synth.make_tiny64(seed=1, S=3000)
    b = synth.make_tiny64(seed=1, S=3000)
    assert _digest(a) == _digest(b)
    assert _digest(a) != _digest(synth.make_tiny64(seed=2, S=3000))
    assert a.N == 2323 and a.M == 8 and a.dims == (64, 64, 64)
    lens = np.diff(a.offsets.numpy())
    assert lens.min() >= 20 and lens.max() <= 200 and a.offsets[0] == 0 and a.offsets[-1] == a.P
    roi = a.roi.numpy()
    assert np.array_equal(roi[roi >= 0], np.arange(a.N))            # raster order
    lab = a.lab.numpy()
    assert set(np.unique(lab)) == set(range(-1, 8))
    # walk step is 0.5 voxel
    p = a.points.numpy()
    seg = p[a.offsets[0]:a.offsets[1]].astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(np.diff(seg, axis=0), axis=1), 0.5, rtol=1e-5)


def test_subject_volumes():
    v = synth.volumes_125mm()
    assert v.dims == (145, 174, 145) and v.M == 70 and 7900 <= v.N <= 8200
    roi = v.roi
    assert np.array_equal(roi[roi >= 0], np.arange(v.N))
    labs = np.unique(v.lab[v.lab >= 0])
    assert np.array_equal(labs, np.arange(70))
    assert not ((v.roi >= 0) & (v.lab >= 0)).any()


def test_subject_walks_stop_at_mask():
    vols = synth.volumes_125mm()
    w = synth.make_125mm(S=3000, vols=vols)
    lens = np.diff(w.offsets.numpy())
    assert lens.min() >= 1 and lens.max() <= 600
    p = w.points.numpy().astype(np.float64)
    c = np.array(vols.centre)
    a = np.array(vols.brain_semi)
    assert (((p - c) / a) ** 2).sum(1).max() <= 1.0 + 1e-6     # every kept point is inside the mask
    assert _digest(w) == _digest(synth.make_125mm(S=3000, vols=vols))


def test_random_small_structure():
    w = synth.random_small(3)
    lens = np.diff(w.offsets.numpy())
    assert (lens == 0).any() and (lens == 1).any()
    assert np.isnan(w.points.numpy()).any()
    assert w.points.dtype == torch.float32 and w.offsets.dtype == torch.int64
