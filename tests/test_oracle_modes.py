"""Pins of the oracle's endpoint modes (Alg. 2 as printed; Alg. 1's seed-to-endpoint count).

Each pin comes from outside the oracle: a hand-worked golden case, an independent dense
brute force (oracle/brute.py), entrywise orderings and identities the definitions force, a
closed form for a straight line, and row sums counted point by point through oracle.voxel.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2302_09247_amd import synth
from tests import _cases

PASS, END, BOTH, SEED = 0, 1, 2, 3
KEYS = {PASS: "C_passthrough", END: "C_end", BOTH: "C_both_ends", SEED: "C_seed_end"}


@pytest.mark.parametrize("mode", [PASS, END, BOTH, SEED])
def test_golden_endpoints(mode):
    g = _cases.load_golden("toy_endpoints.json")
    C = oracle.count(g["points"], g["offsets"], g["roi"], g["lab"], g["N"], g["M"], mode=mode)
    np.testing.assert_array_equal(C, g[KEYS[mode]])


def test_golden_two_streamlines_endpoint_modes():
    # both streamlines of the first toy case end outside every label, and neither starts in the ROI:
    # only the both-ends mode counts (A starts on label 0, B on label 2); worked by hand from its notes
    g = _cases.load_golden("toy_two_streamlines.json")
    args = (g["points"], g["offsets"], g["roi"], g["lab"], g["N"], g["M"])
    assert not oracle.count(*args, mode=END).any()
    assert not oracle.count(*args, mode=SEED).any()
    np.testing.assert_array_equal(oracle.count(*args, mode=BOTH), [[1, 0, 0], [1, 0, 1], [1, 0, 0]])


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("mode", [END, BOTH, SEED])
def test_equals_brute_force(seed, mode):
    w = synth.random_small(seed, N=(None if seed % 2 else 6), bad_values=bool(seed % 3 == 0))
    args = (w.points.numpy(), w.offsets.numpy(), w.roi.numpy(), w.lab.numpy(), w.N, w.M)
    for scale in (1.0, 1.7857143):
        np.testing.assert_array_equal(oracle.count(*args, scale=scale, mode=mode),
                                      brute.brute_count_ends(*args, scale=scale, mode=mode))


def _tiny():
    w = synth.make_tiny64(seed=7, S=1500)
    return w, (w.points.numpy(), w.offsets.numpy(), w.roi.numpy(), w.lab.numpy(), w.N, w.M)


def test_entrywise_orderings():
    w, args = _tiny()
    P, E, B, Sd = (oracle.count(*args, mode=m) for m in (PASS, END, BOTH, SEED))
    assert np.all(Sd <= E) and np.all(E <= B) and np.all(B <= P)
    assert E.sum() > 0 and Sd.sum() > 0 and (B - E).sum() > 0 and (P - B).sum() > 0


def test_reversal_identity():
    # reversing a streamline swaps its ends: END(L) + END(reversed L) - BOTH(L) counts, per
    # streamline, its rows at the label shared by both ends (zero when the end labels differ)
    w, (pts, off, roi, lab, N, M) = _tiny()
    rev_pts = pts[::-1].copy()
    rev_off = (off[-1] - off[::-1]).copy()
    E = oracle.count(pts, off, roi, lab, N, M, mode=END)
    Er = oracle.count(rev_pts, rev_off, roi, lab, N, M, mode=END)
    B = oracle.count(pts, off, roi, lab, N, M, mode=BOTH)
    np.testing.assert_array_equal(oracle.count(rev_pts, rev_off, roi, lab, N, M, mode=BOTH), B)
    Z, Y, X = roi.shape
    same = np.zeros((N, M), np.int64)
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        if b <= a:
            continue
        lf, ll = oracle.voxel(pts[a], (X, Y, Z)), oracle.voxel(pts[b - 1], (X, Y, Z))
        mf = lab.reshape(-1)[lf] if lf >= 0 else -1
        ml = lab.reshape(-1)[ll] if ll >= 0 else -1
        if mf == ml and 0 <= ml < M:
            rows = {int(roi.reshape(-1)[v]) for v in (oracle.voxel(p, (X, Y, Z)) for p in pts[a:b])
                    if v >= 0 and 0 <= roi.reshape(-1)[v] < N}
            for r in rows:
                same[r, ml] += 1
    np.testing.assert_array_equal(E + Er - B, same)


def test_seed_end_row_sums():
    # row i of the seed-to-endpoint matrix sums to the streamlines whose first point is in row i
    # and whose last point has a label, counted here one streamline at a time
    w, (pts, off, roi, lab, N, M) = _tiny()
    Z, Y, X = roi.shape
    want = np.zeros(N, np.int64)
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        if b <= a:
            continue
        vf, vl = oracle.voxel(pts[a], (X, Y, Z)), oracle.voxel(pts[b - 1], (X, Y, Z))
        if vf >= 0 and vl >= 0 and 0 <= roi.reshape(-1)[vf] < N and 0 <= lab.reshape(-1)[vl] < M:
            want[roi.reshape(-1)[vf]] += 1
    np.testing.assert_array_equal(oracle.count(pts, off, roi, lab, N, M, mode=SEED).sum(axis=1), want)


def test_straight_line_closed_form():
    # a line along x through voxels 0..9 of row y=1; ROI rows = x for x in 2..6; labels at x=0 (3)
    # and x=9 (5).  End mode: rows 2..6 x label 5; both ends: also label 3; seed: none (x=0 not ROI);
    # starting the line at x=2 instead makes the seed row 2.
    X, Y, Z = 10, 3, 1
    roi = np.full((Z, Y, X), -1, np.int32)
    lab = np.full((Z, Y, X), -1, np.int32)
    roi[0, 1, 2:7] = np.arange(5)
    lab[0, 1, 0], lab[0, 1, 9] = 3, 5
    for x0, seed_row in ((0.0, None), (2.0, 0)):
        pts = np.stack([np.arange(x0, 9.01, 0.5), np.ones_like(np.arange(x0, 9.01, 0.5)),
                        np.zeros_like(np.arange(x0, 9.01, 0.5))], axis=1).astype(np.float32)
        off = np.array([0, len(pts)], np.int64)
        E = oracle.count(pts, off, roi, lab, 5, 6, mode=END)
        want = np.zeros((5, 6), np.int64)
        want[:, 5] = 1
        np.testing.assert_array_equal(E, want)
        B = oracle.count(pts, off, roi, lab, 5, 6, mode=BOTH)
        if x0 == 0.0:
            want[:, 3] = 1
        np.testing.assert_array_equal(B, want)
        Sd = oracle.count(pts, off, roi, lab, 5, 6, mode=SEED)
        want = np.zeros((5, 6), np.int64)
        if seed_row is not None:
            want[seed_row, 5] = 1
        np.testing.assert_array_equal(Sd, want)


def test_chunked_modes_are_additive():
    w, args = _tiny()
    for mode in (END, BOTH, SEED):
        np.testing.assert_array_equal(oracle.count_chunked(*args, mode=mode, streamlines_per_chunk=97),
                                      oracle.count(*args, mode=mode))
