"""Pins of the oracle's upsampled pass-through count (Section 3, super-resolving connectivity
features): a hand-worked golden case for u = 1..4, u = 1 being the plain count, an independent
numpy densification counted by the brute force, inclusion orderings the construction forces
(the points for u are among those for 2u), and a coarse straight line that upsampling fills in."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2302_09247_amd import synth
from tests import _cases


@pytest.mark.parametrize("u", [1, 2, 3, 4])
def test_golden(u):
    g = _cases.load_golden("toy_upsample.json")
    np.testing.assert_array_equal(
        oracle.count(g["points"], g["offsets"], g["roi"], g["lab"], g["N"], g["M"], upsample=u), g[f"C_u{u}"])


@pytest.mark.parametrize("seed", range(6))
def test_u1_is_the_plain_count(seed):
    w = synth.random_small(seed, bad_values=True)
    args = (w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    for scale in (1.0, 1.7857143):
        np.testing.assert_array_equal(oracle.count(*args, scale=scale, upsample=1), oracle.count(*args, scale=scale))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("u", [2, 3, 4])
def test_equals_numpy_densification(seed, u):
    w = synth.random_small(seed, N=(None if seed % 2 else 6), bad_values=bool(seed % 3 == 0))
    for scale in (1.0, 1.7857143):
        pts, off = brute.brute_upsample(w.points.numpy(), w.offsets.numpy(), scale, u)
        want = brute.brute_count(pts, off, w.roi.numpy(), w.lab.numpy(), w.N, w.M, scale=1.0)
        got = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=scale, upsample=u)
        np.testing.assert_array_equal(got, want)


def test_inclusion_orderings():
    # the points for u are among those for 2u (a_{2t} = fl32(2t/2u) = a_t), and the original points
    # are among every u: C(1) <= C(2) <= C(4) and C(1) <= C(3) entrywise
    w = synth.make_tiny64(seed=11, S=800)
    args = (w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    C1, C2, C3, C4 = (oracle.count(*args, upsample=u, scale=1.7857143) for u in (1, 2, 3, 4))
    assert np.all(C1 <= C2) and np.all(C2 <= C4) and np.all(C1 <= C3)
    assert (C4 - C1).sum() > 0


def test_coarse_line_filled_in():
    # a straight line along x with 2-voxel steps touches every other voxel; u = 4 (0.5-voxel
    # spacing) touches all of them, giving the closed form of the line case
    dims, M = (21, 3, 3), 3
    lab_of = lambda x, y, z: x % 3 if x in (0, 20) else -1   # noqa: E731
    pts_fine, off_fine, roi, lab, N, M, C_fine = _cases.line_case((0.0, 1.0, 1.0), (0.5, 0.0, 0.0), 41, dims, M, lab_of)
    coarse = pts_fine[::4].copy()   # x = 0, 2, 4, ..., 20
    off = np.array([0, coarse.shape[0]], np.int64)
    C1 = oracle.count(coarse, off, roi, lab, N, M)
    C4 = oracle.count(coarse, off, roi, lab, N, M, upsample=4)
    np.testing.assert_array_equal(C4, C_fine)
    assert C1.sum() < C4.sum()


def test_upsample_needs_passthrough():
    w = synth.random_small(1)
    with pytest.raises(ValueError):
        oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, mode=1, upsample=2)
