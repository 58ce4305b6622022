"""Pins of the CPU oracle against facts the paper and the mathematics fix.

The oracle computes the pass-through matrix of FastCod Section 2 (Alg. 2).  The paper
prints no numeric example (its toy example is a figure), so the pins are: a hand-worked
toy case, exact voxel sets of straight streamlines, IEEE binary32 rounding facts, brute
force on tiny inputs, invariants, and special cases that reduce to textbook routines.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import brute
from paper_2302_09247_amd import synth
from tests import _cases


def test_golden_toy_two_streamlines():
    g = _cases.load_golden("toy_two_streamlines.json")
    C = oracle.count(g["points"], g["offsets"], g["roi"], g["lab"], g["N"], g["M"])
    np.testing.assert_array_equal(C, g["C"])


@pytest.mark.parametrize("value,X,expected", _cases.ROUNDING_PINS)
def test_rounding_pins(value, X, expected):
    for axis in range(3):
        dims = [3, 3, 3]
        dims[axis] = X
        p = [1.0, 1.0, 1.0]
        p[axis] = value
        got = oracle.voxel(p, dims)
        if expected < 0:
            assert got == -1
        else:
            v = [1, 1, 1]
            v[axis] = expected
            assert got == v[0] + dims[0] * (v[1] + dims[1] * v[2])


def test_rounding_pins_brute_agrees():
    for value, X, expected in _cases.ROUNDING_PINS:
        v, inside = brute.brute_voxel([[value, 1.0, 1.0]], (X, 3, 3))
        assert bool(inside[0]) == (expected >= 0)
        if expected >= 0:
            assert v[0, 0] == expected


LINES = [
    # origin, step, T, dims, M
    ((0.25, 2.0, 1.0), (0.5, 0.0, 0.0), 23, (13, 4, 3), 4),
    ((1.0, -0.25, 2.0), (0.0, 0.5, 0.0), 17, (3, 9, 4), 3),
    ((1.0, 2.0, -0.75), (0.0, 0.0, 0.5), 21, (3, 4, 10), 5),
    ((0.125, 0.375, 0.0625), (0.25, 0.25, 0.25), 40, (11, 12, 13), 6),
    ((9.875, 0.375, 11.0625), (-0.25, 0.25, -0.25), 44, (11, 12, 13), 6),
    ((-3.0, 1.0, 1.0), (0.75, 0.125, 0.0), 30, (12, 6, 3), 3),   # enters the grid from outside
]


def _label_of(M):
    return lambda x, y, z: ((x + 2 * y + 3 * z) % (M + 1)) - 1   # -1 on some voxels


@pytest.mark.parametrize("origin,step,T,dims,M", LINES)
def test_closed_form_straight_lines(origin, step, T, dims, M):
    pts, off, roi, lab, N, M, Cexp = _cases.line_case(origin, step, T, dims, M, _label_of(M))
    C = oracle.count(pts, off, roi, lab, N, M)
    np.testing.assert_array_equal(C, Cexp)


def test_closed_form_several_lines_sum():
    parts = [_cases.line_case(o, s, T, (11, 12, 13), 6, _label_of(6)) for (o, s, T, d, m) in LINES[3:5]]
    pts = np.concatenate([p[0] for p in parts])
    off = np.array([0, parts[0][0].shape[0], pts.shape[0]], dtype=np.int64)
    C = oracle.count(pts, off, parts[0][2], parts[0][3], parts[0][4], 6)
    np.testing.assert_array_equal(C, parts[0][6] + parts[1][6])


def test_scale_two_closed_form():
    # p*2 is exact for these dyadic coordinates, so the scaled line is the line with double step
    pts, off, roi, lab, N, M, Cexp = _cases.line_case((0.25, 2.0, 1.0), (1.0, 0.0, 0.0), 12, (25, 5, 3), 4,
                                                      _label_of(4))
    half = (pts / np.float32(2.0)).astype(np.float32)
    C = oracle.count(half, off, roi, lab, N, M, scale=2.0)
    np.testing.assert_array_equal(C, Cexp)


@pytest.mark.parametrize("seed", range(12))
def test_oracle_equals_brute_force(seed):
    w = synth.random_small(seed, N=(None if seed % 3 else 6), bad_values=(seed % 2 == 0),
                           dims=[(12, 10, 9), (7, 16, 5), (20, 3, 4)][seed % 3])
    args = (w.points.numpy(), w.offsets.numpy(), w.roi.numpy(), w.lab.numpy(), w.N, w.M)
    for scale in (1.0, 1.7857143):
        np.testing.assert_array_equal(oracle.count(*args, scale=scale), brute.brute_count(*args, scale=scale))


@settings(max_examples=40, deadline=None)
@given(seed=st.integers(0, 10 ** 6), X=st.integers(1, 9), Y=st.integers(1, 9), Z=st.integers(1, 9),
       S=st.integers(0, 12), M=st.integers(1, 6), N=st.integers(1, 12))
def test_oracle_equals_brute_force_hypothesis(seed, X, Y, Z, S, M, N):
    w = synth.random_small(seed, dims=(X, Y, Z), S=S, N=N, M=M, max_len=25, bad_values=bool(seed % 2))
    args = (w.points.numpy(), w.offsets.numpy(), w.roi.numpy(), w.lab.numpy(), w.N, w.M)
    np.testing.assert_array_equal(oracle.count(*args), brute.brute_count(*args))


def _sets(w, scale=1.0):
    """Per-streamline sets via the brute-force voxel lookup (independent of the C oracle)."""
    pts, off = w.points.numpy(), w.offsets.numpy()
    roi, lab = w.roi.numpy(), w.lab.numpy()
    Z, Y, X = roi.shape
    out = []
    for s in range(w.S):
        v, ins = brute.brute_voxel(pts[off[s]:off[s + 1]], (X, Y, Z), scale)
        v = v[ins]
        r = roi[v[:, 2], v[:, 1], v[:, 0]]
        m = lab[v[:, 2], v[:, 1], v[:, 0]]
        out.append((np.unique(r[(r >= 0) & (r < w.N)]), np.unique(m[(m >= 0) & (m < w.M)])))
    return out


def test_invariants_tiny64():
    w = synth.make_tiny64(seed=11, S=1500)
    C = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    sets = _sets(w)
    visits_i = np.zeros(w.N, np.int64)
    visits_m = np.zeros(w.M, np.int64)
    total = 0
    rowsum = np.zeros(w.N, np.int64)
    for I, L in sets:
        visits_i[I] += 1
        visits_m[L] += 1
        total += I.size * L.size
        rowsum[I] += L.size
    assert (C <= visits_i[:, None]).all() and (C <= visits_m[None, :]).all()
    assert C.sum() == total
    np.testing.assert_array_equal(C.sum(1), rowsum)
    assert total > 0


def _subset(w, idx):
    pts, off = w.points.numpy(), w.offsets.numpy()
    parts = [pts[off[s]:off[s + 1]] for s in idx]
    P = np.concatenate(parts) if parts else np.zeros((0, 3), np.float32)
    o = np.zeros(len(parts) + 1, np.int64)
    o[1:] = np.cumsum([p.shape[0] for p in parts])
    return P, o


def test_additivity_and_permutation():
    w = synth.make_tiny64(seed=5, S=800)
    rng = np.random.default_rng(0)
    roi, lab = w.roi.numpy(), w.lab.numpy()
    full = oracle.count(w.points, w.offsets, roi, lab, w.N, w.M)
    perm = rng.permutation(w.S)
    a, b = perm[:300], perm[300:]
    Ca = oracle.count(*_subset(w, a), roi, lab, w.N, w.M)
    Cb = oracle.count(*_subset(w, b), roi, lab, w.N, w.M)
    np.testing.assert_array_equal(Ca + Cb, full)
    np.testing.assert_array_equal(oracle.count(*_subset(w, perm), roi, lab, w.N, w.M), full)
    np.testing.assert_array_equal(oracle.count_chunked(w.points, w.offsets, roi, lab, w.N, w.M,
                                                       streamlines_per_chunk=97, workers=3), full)


def test_reverse_shuffle_duplicate_points():
    w = synth.make_tiny64(seed=6, S=600)
    pts, off = w.points.numpy(), w.offsets.numpy()
    roi, lab = w.roi.numpy(), w.lab.numpy()
    full = oracle.count(pts, off, roi, lab, w.N, w.M)
    rng = np.random.default_rng(1)
    rev, shuf, dup, doff = [], [], [], [0]
    for s in range(w.S):
        seg = pts[off[s]:off[s + 1]]
        rev.append(seg[::-1])
        shuf.append(seg[rng.permutation(seg.shape[0])])
        d = np.repeat(seg, rng.integers(1, 4, size=seg.shape[0]), axis=0)
        dup.append(d)
        doff.append(doff[-1] + d.shape[0])
    np.testing.assert_array_equal(oracle.count(np.concatenate(rev), off, roi, lab, w.N, w.M), full)
    np.testing.assert_array_equal(oracle.count(np.concatenate(shuf), off, roi, lab, w.N, w.M), full)
    np.testing.assert_array_equal(oracle.count(np.concatenate(dup), np.array(doff), roi, lab, w.N, w.M), full)


def test_role_swap_symmetry():
    # pass-through for both volumes: exchanging the ROI and target volumes transposes C
    rng = np.random.default_rng(3)
    w = synth.random_small(4, dims=(10, 11, 12), S=60, N=9, M=7)
    A = w.roi.numpy()
    B = w.lab.numpy()
    args = (w.points.numpy(), w.offsets.numpy())
    C_ab = oracle.count(*args, A, B, 9, 7)
    C_ba = oracle.count(*args, B, A, 7, 9)
    np.testing.assert_array_equal(C_ab, C_ba.T)
    assert C_ab.sum() > 0
    del rng


def test_single_streamline_is_rank_one():
    w = synth.make_tiny64(seed=2, S=50)
    roi, lab = w.roi.numpy(), w.lab.numpy()
    for s in range(w.S):
        C = oracle.count(*_subset(w, [s]), roi, lab, w.N, w.M)
        assert set(np.unique(C)) <= {0, 1}
        if C.any():
            rows = np.flatnonzero(C.any(1))
            cols = np.flatnonzero(C.any(0))
            np.testing.assert_array_equal(C[np.ix_(rows, cols)], 1)
            assert C.sum() == rows.size * cols.size


def test_one_label_everywhere_is_visit_count():
    # lab == 0 on every voxel (M = 1): C[:, 0] = number of streamlines that visit ROI row i,
    # i.e. a bincount of each streamline's unique ROI rows among its in-grid points
    w = synth.make_tiny64(seed=9, S=700)
    roi = w.roi.numpy()
    lab = np.zeros_like(roi)
    C = oracle.count(w.points, w.offsets, roi, lab, w.N, 1)
    counts = np.zeros(w.N, np.int64)
    pts, off = w.points.numpy(), w.offsets.numpy()
    Z, Y, X = roi.shape
    for s in range(w.S):
        seg = pts[off[s]:off[s + 1]].astype(np.float64)
        f = np.floor(seg + 0.5)   # exact here: |p| < 2^20, so float64 adds no rounding
        ok = np.all((f >= 0) & (f < np.array([X, Y, Z])), axis=1)
        v = f[ok].astype(np.int64)
        r = roi[v[:, 2], v[:, 1], v[:, 0]]
        counts += np.bincount(np.unique(r[r >= 0]), minlength=w.N)
    np.testing.assert_array_equal(C[:, 0], counts)


def test_scale_one_is_identity_and_empty_inputs():
    w = synth.random_small(8)
    args = (w.points.numpy(), w.offsets.numpy(), w.roi.numpy(), w.lab.numpy(), w.N, w.M)
    np.testing.assert_array_equal(oracle.count(*args, scale=1.0), oracle.count(*args))
    C0 = oracle.count(np.zeros((0, 3), np.float32), np.zeros(1, np.int64), w.roi, w.lab, w.N, w.M)
    assert C0.shape == (w.N, w.M) and not C0.any()
    Ce = oracle.count(np.zeros((0, 3), np.float32), np.zeros(5, np.int64), w.roi, w.lab, w.N, w.M)
    assert not Ce.any()
