"""The GPU parity cases must exercise the pair path: a case whose exact C is all zero only shows that
nothing spurious is counted.  Checked here on the CPU, with the oracle, for the generators those
cases draw from (no GPU)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth


def _pairs(w, mode=0):
    return int(oracle.count(w.points.numpy(), w.offsets.numpy(), np.asarray(w.roi), np.asarray(w.lab),
                            w.N, w.M, w.scale, mode=mode).sum())


@pytest.mark.parametrize("seed", [1, 4, 8])
def test_tiny64_cases_produce_pairs_in_both_modes(seed):
    w = synth.make_tiny64(seed=seed, S=3000)
    assert _pairs(w) > 1000
    assert _pairs(w, mode=1) > 100


@pytest.mark.parametrize("seed", range(0, 16, 3))
def test_random_small_cases_produce_pairs(seed):
    assert _pairs(synth.random_small(seed)) > 50


def test_interleaved_volume_gives_short_walks_pairs():
    vols = synth.volumes_interleaved64()
    # ROI voxels and labels alternate in 4-voxel cubes: disjoint, both numerous, ROI numbered in
    # raster order
    assert ((vols.roi >= 0) & (vols.lab >= 0)).sum() == 0
    assert vols.N == int((vols.roi >= 0).sum()) > 50_000
    np.testing.assert_array_equal(vols.roi[vols.roi >= 0], np.arange(vols.N))
    assert set(np.unique(vols.lab[vols.lab >= 0])) == set(range(8))
    g = torch.Generator().manual_seed(5)
    n = 20_000
    seeds = synth.uniform_in_ellipsoid(n, (32.0, 32.0, 32.0), (30.0, 30.0, 30.0), g, "cpu")
    pts, L = synth.random_walks(n, seeds, torch.randint(1, 13, (n,), generator=g), g, None)
    off = np.concatenate([[0], np.cumsum(L.numpy())]).astype(np.int64)
    C = oracle.count(pts.numpy(), off, vols.roi, vols.lab, vols.N, vols.M)
    assert C.sum() > 10_000
    # the shell volume, by contrast, is out of reach of walks this short
    tiny = synth.volumes_tiny64()
    assert oracle.count(pts.numpy(), off, tiny.roi, tiny.lab, tiny.N, tiny.M).sum() == 0
