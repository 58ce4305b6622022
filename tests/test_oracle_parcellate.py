"""Pins of the oracle's parcellation outputs (Section 3, 'Pie-glyphs'): hand-worked rows, the
exact rational fraction within half a float ulp (plus the double rounding step), invariance under
scaling C and permuting rows, and the definitions' consequences on random matrices."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "parcellation_rows.json")


def _ulp32(x: float) -> Fraction:
    """Spacing of float32 numbers at |x| (exact)."""
    x = abs(float(x))
    if x == 0.0:
        return Fraction(2) ** -149
    e = int(np.floor(np.log2(x)))
    if Fraction(2) ** (e + 1) <= Fraction(x):
        e += 1
    if Fraction(2) ** e > Fraction(x):
        e -= 1
    return Fraction(2) ** max(e - 23, -149)


def _close_to_rational(f: np.float32, q: Fraction) -> bool:
    # round to float32 of q taken through double: at most half a float ulp plus one double rounding
    err = abs(Fraction(float(f)) - q)
    return err <= _ulp32(float(q)) / 2 + abs(q) * Fraction(2) ** -52


def test_golden_rows():
    g = json.load(open(GOLDEN))
    label, frac, sums = oracle.parcellate(np.array(g["C"]))
    np.testing.assert_array_equal(label, g["labels"])
    np.testing.assert_array_equal(sums, g["sums"])
    for i, row in enumerate(g["fractions"]):
        for m, txt in enumerate(row):
            q = Fraction(txt)
            assert _close_to_rational(frac[i, m], q), (i, m, frac[i, m], txt)
            if q.denominator & (q.denominator - 1) == 0:   # dyadic: exactly representable
                assert Fraction(float(frac[i, m])) == q


@pytest.mark.parametrize("seed", range(4))
def test_fractions_against_exact_rationals(seed):
    rng = np.random.default_rng(seed)
    hi = [10, 1000, 1 << 20, 1 << 26][seed]   # counts above 2^24 are inexact in float32
    C = rng.integers(0, hi, size=(60, 37)).astype(np.int64)
    C[rng.random(C.shape) < 0.5] = 0
    C[3] = 0
    label, frac, sums = oracle.parcellate(C)
    for i in range(C.shape[0]):
        s = int(C[i].sum())
        assert sums[i] == s
        if s == 0:
            assert label[i] == -1 and not frac[i].any()
            continue
        mx = int(C[i].max())
        assert C[i, label[i]] == mx and all(C[i, m] < mx for m in range(label[i]))
        for m in range(C.shape[1]):
            assert _close_to_rational(frac[i, m], Fraction(int(C[i, m]), s)), (i, m)


def test_scale_and_permutation_invariance():
    rng = np.random.default_rng(9)
    C = rng.integers(0, 50, size=(40, 23)).astype(np.int64)
    C[rng.random(C.shape) < 0.6] = 0
    l1, f1, s1 = oracle.parcellate(C)
    l3, f3, s3 = oracle.parcellate(3 * C)   # the same rationals: bit-identical fractions
    np.testing.assert_array_equal(l1, l3)
    np.testing.assert_array_equal(f1.view(np.uint32), f3.view(np.uint32))
    np.testing.assert_array_equal(3 * s1, s3)
    perm = rng.permutation(C.shape[0])
    lp, fp, sp = oracle.parcellate(C[perm])
    np.testing.assert_array_equal(lp, l1[perm])
    np.testing.assert_array_equal(fp, f1[perm])


def test_fractions_sum_to_one():
    rng = np.random.default_rng(5)
    C = rng.integers(0, 1000, size=(100, 180)).astype(np.int64)
    _, frac, sums = oracle.parcellate(C)
    tot = frac.astype(np.float64).sum(axis=1)
    assert np.all(np.abs(tot - 1.0) <= 180 * 2.0 ** -24)


def test_empty_matrix_rows():
    label, frac, sums = oracle.parcellate(np.zeros((0, 5), np.int64))
    assert label.shape == (0,) and frac.shape == (0, 5)
