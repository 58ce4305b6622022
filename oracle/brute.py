"""Brute-force connectivity matrix in numpy -- TEST INFRASTRUCTURE ONLY.

Second, independent CPU implementation of the FastCod pass-through matrix
(Section 2 "Method", Alg. 2), for tiny inputs.  It forms, per streamline l,
the dense 0/1 vectors h_l in {0,1}^N (ROI rows passed through) and
g_l in {0,1}^M (target labels passed through) and sums their outer products:
C = sum_l h_l g_l^T.  Voxels are looked up as roi[z, y, x] with 3-D indexing,
never through a linear index, so a mistake in the C oracle's index formula
cannot be repeated here.  All coordinate arithmetic stays in float32.
"""
from __future__ import annotations

import numpy as np


def brute_voxel(p, dims, scale: float = 1.0):
    """(x, y, z) voxel of each point of p [K,3] and a mask of points inside the grid."""
    p = np.asarray(p, dtype=np.float32).reshape(-1, 3)
    with np.errstate(invalid="ignore", over="ignore"):
        q = p * np.float32(scale)
        f = np.floor(q + np.float32(0.5))
        dims_f = np.asarray(dims, dtype=np.float64)
        inside = np.all(f >= 0, axis=1) & np.all(f.astype(np.float64) < dims_f, axis=1)
    v = np.zeros((p.shape[0], 3), dtype=np.int64)
    v[inside] = f[inside].astype(np.int64)
    return v, inside


def brute_count(points, offsets, roi, lab, N: int, M: int, scale: float = 1.0) -> np.ndarray:
    points = np.asarray(points, dtype=np.float32).reshape(-1, 3)
    offsets = np.asarray(offsets, dtype=np.int64)
    roi = np.asarray(roi, dtype=np.int32)
    lab = np.asarray(lab, dtype=np.int32)
    Z, Y, X = roi.shape
    C = np.zeros((N, M), dtype=np.int64)
    for s in range(offsets.shape[0] - 1):
        v, inside = brute_voxel(points[offsets[s]:offsets[s + 1]], (X, Y, Z), scale)
        v = v[inside]
        r = roi[v[:, 2], v[:, 1], v[:, 0]]
        m = lab[v[:, 2], v[:, 1], v[:, 0]]
        h = np.zeros(N, dtype=np.int64)
        g = np.zeros(M, dtype=np.int64)
        h[r[(r >= 0) & (r < N)]] = 1
        g[m[(m >= 0) & (m < M)]] = 1
        C += np.outer(h, g)
    return C


def brute_count_ends(points, offsets, roi, lab, N: int, M: int, scale: float = 1.0, mode: int = 1) -> np.ndarray:
    """The endpoint modes as dense outer products, for tiny inputs.

    mode 1 (Alg. 2 as printed): h_l = ROI rows passed through, g_l = one-hot label of the last point.
    mode 2: g_l = labels of the first and the last point (0/1 entries, so a shared label counts once).
    mode 3 (Alg. 1's count): h_l = one-hot row of the first point (the seed), g_l as in mode 1.
    """
    points = np.asarray(points, dtype=np.float32).reshape(-1, 3)
    offsets = np.asarray(offsets, dtype=np.int64)
    roi = np.asarray(roi, dtype=np.int32)
    lab = np.asarray(lab, dtype=np.int32)
    Z, Y, X = roi.shape
    C = np.zeros((N, M), dtype=np.int64)
    for s in range(offsets.shape[0] - 1):
        seg = points[offsets[s]:offsets[s + 1]]
        if seg.shape[0] == 0:
            continue
        v, inside = brute_voxel(seg, (X, Y, Z), scale)
        r = np.where(inside, roi[v[:, 2], v[:, 1], v[:, 0]], -1)
        m = np.where(inside, lab[v[:, 2], v[:, 1], v[:, 0]], -1)
        h = np.zeros(N, dtype=np.int64)
        g = np.zeros(M, dtype=np.int64)
        rows = r[:1] if mode == 3 else r
        h[rows[(rows >= 0) & (rows < N)]] = 1
        ends = m[[0, -1]] if mode == 2 else m[-1:]
        g[ends[(ends >= 0) & (ends < M)]] = 1
        C += np.outer(h, g)
    return C


def brute_upsample(points, offsets, scale: float, u: int):
    """Scaled, upsampled streamlines as (points [P', 3] float32, offsets): u - 1 points
    q_k + a_t (q_{k+1} - q_k), a_t = t/u, inserted between neighbours, every step a float32
    operation of numpy (no fused multiply-add).  Count the result with scale 1."""
    points = np.asarray(points, dtype=np.float32).reshape(-1, 3)
    offsets = np.asarray(offsets, dtype=np.int64)
    out, off = [], [0]
    err = np.seterr(invalid="ignore", over="ignore")   # NaN / inf coordinates stay NaN / inf
    for s in range(offsets.shape[0] - 1):
        q = points[offsets[s]:offsets[s + 1]] * np.float32(scale)
        seq = []
        for k in range(q.shape[0]):
            seq.append(q[k])
            if k + 1 < q.shape[0]:
                d = q[k + 1] - q[k]
                for t in range(1, u):
                    a = np.float32(t) / np.float32(u)
                    seq.append(q[k] + a * d)
        arr = np.array(seq, dtype=np.float32).reshape(-1, 3)
        out.append(arr)
        off.append(off[-1] + arr.shape[0])
    np.seterr(**err)
    pts = np.concatenate(out) if out else np.zeros((0, 3), np.float32)
    return pts, np.array(off, dtype=np.int64)
