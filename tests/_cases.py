"""Hand-built cases shared by the CPU (oracle) and GPU (parity) tests.

Every expected value here is derived by exact integer / rational arithmetic from the
definition of the pass-through matrix (FastCod Section 2, Alg. 2), never by running
either implementation.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name: str):
    with open(os.path.join(GOLDEN, name)) as f:
        g = json.load(f)
    X, Y, Z = g["dims"]
    roi = np.full((Z, Y, X), -1, dtype=np.int32)
    lab = np.full((Z, Y, X), -1, dtype=np.int32)
    for x, y, z, v in g["roi_voxels"]:
        roi[z, y, x] = v
    for x, y, z, v in g["label_voxels"]:
        lab[z, y, x] = v
    pts, off = [], [0]
    for s in g["streamlines"]:
        arr = np.array([[float(c) for c in p] for p in s], dtype=np.float32).reshape(-1, 3)
        pts.append(arr)
        off.append(off[-1] + arr.shape[0])
    points = np.concatenate(pts) if pts else np.zeros((0, 3), np.float32)
    out = dict(points=points, offsets=np.array(off, dtype=np.int64), roi=roi, lab=lab, N=g["N"], M=g["M"])
    for k, v in g.items():
        if k == "C" or k.startswith("C_"):
            out[k] = np.array(v, dtype=np.int64)
    return out


def identity_volumes(dims, M, label_of):
    """ROI row = linear voxel index for every voxel (N = X*Y*Z); lab[z,y,x] = label_of(x,y,z)
    (an int in [0,M) or -1)."""
    X, Y, Z = dims
    roi = np.arange(X * Y * Z, dtype=np.int32).reshape(Z, Y, X)
    lab = np.full((Z, Y, X), -1, dtype=np.int32)
    for z in range(Z):
        for y in range(Y):
            for x in range(X):
                lab[z, y, x] = label_of(x, y, z)
    return roi, lab


def exact_voxel(coord: Fraction) -> int:
    """floor(c + 1/2) in exact arithmetic (valid when c + 1/2 is exactly representable)."""
    return math.floor(coord + Fraction(1, 2))


def line_case(origin, step, T, dims, M, label_of):
    """One straight streamline p_t = origin + t*step (dyadic values, so float32 is exact).

    Returns (points, offsets, roi, lab, N, M, C_expected) with C derived from the exact voxel
    set: C[i][m] = 1 iff voxel i is visited and label m is seen on a visited voxel."""
    X, Y, Z = dims
    roi, lab = identity_volumes(dims, M, label_of)
    pts = []
    visited = set()
    for t in range(T):
        c = [Fraction(origin[k]) + t * Fraction(step[k]) for k in range(3)]
        pts.append([float(v) for v in c])
        v = [exact_voxel(c[k]) for k in range(3)]
        if all(0 <= v[k] < dims[k] for k in range(3)):
            visited.add(tuple(v))
    points = np.array(pts, dtype=np.float32)
    for t in range(T):   # the case is only valid if float32 holds every coordinate exactly
        assert all(Fraction(float(points[t, k])) == Fraction(origin[k]) + t * Fraction(step[k]) for k in range(3))
    N = X * Y * Z
    rows = sorted(x + X * (y + Y * z) for (x, y, z) in visited)
    labels = sorted({label_of(*v) for v in visited} - {-1})
    C = np.zeros((N, M), dtype=np.int64)
    for i in rows:
        for m in labels:
            C[i, m] = 1
    return points, np.array([0, T], dtype=np.int64), roi, lab, N, M, C


# (value, X, expected voxel or -1), IEEE binary32 facts:
#   0.49999997f = 0.5 - 2^-25; fl32(0.49999997f + 0.5f) is a tie between 1 - 2^-24 and 1 and
#   rounds to the even significand, 1.0, so the voxel is 1 (exact real arithmetic would give 0).
ROUNDING_PINS = [
    (0.0, 64, 0),
    (0.49999994, 64, 0),      # 0.5 - 2^-24: sum 1 - 2^-24 is representable -> floor 0
    (0.49999997, 64, 1),      # 0.5 - 2^-25: tie, rounds to 1.0 -> voxel 1
    (0.5, 64, 1),
    (1.4999999, 64, 1),
    (1.5, 64, 2),
    (-0.5, 64, 0),            # -0.5 + 0.5 = +0 -> voxel 0 (inside)
    (-0.49999997, 64, 0),
    (-0.50000006, 64, -1),    # sum is -2^-24 < 0 -> outside
    (63.499996, 64, 63),      # nextafter(63.5, 0) -> 63.999996 -> 63
    (63.5, 64, -1),           # X - 0.5 -> 64 = X -> outside
    (float("nan"), 64, -1),
    (float("inf"), 64, -1),
    (float("-inf"), 64, -1),
    (1e30, 64, -1),
    (-1e30, 64, -1),
    (16777215.0, 2 ** 25, 16777216),   # 2^24 - 1 + 0.5 is a tie -> rounds to 2^24 (even)
]
