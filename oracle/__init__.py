"""CPU oracle for pass-through connectivity counting -- TEST INFRASTRUCTURE ONLY.

Two independent CPU implementations of the FastCod connectivity matrix
(Section 2 "Method", Alg. 2: passthrough, loc2region and the C update):

* ``oracle.c`` (plain C, loaded with ctypes): the definition written out, one
  streamline at a time, with sort/unique set semantics.  ``count`` below.
* ``brute.py`` (numpy): dense 0/1 hit vectors and a sum of outer products,
  used to pin the C oracle on tiny inputs.  ``brute_count`` below.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library and
imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .brute import brute_count, brute_count_ends, brute_voxel  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_voxel.restype = ctypes.c_int64
        lib.oracle_voxel.argtypes = [ctypes.c_float] * 4 + [ctypes.c_void_p]
        common = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_int32, ctypes.c_int32, ctypes.c_float]
        lib.oracle_count.restype = ctypes.c_int
        lib.oracle_count.argtypes = common + [ctypes.c_void_p]
        lib.oracle_count_endpoint.restype = ctypes.c_int
        lib.oracle_count_endpoint.argtypes = common + [ctypes.c_int, ctypes.c_void_p]
        lib.oracle_count_seed_endpoint.restype = ctypes.c_int
        lib.oracle_count_seed_endpoint.argtypes = common + [ctypes.c_void_p]
        lib.oracle_count_upsampled.restype = ctypes.c_int
        lib.oracle_count_upsampled.argtypes = common + [ctypes.c_int32, ctypes.c_void_p]
        lib.oracle_parcellate.restype = ctypes.c_int
        lib.oracle_parcellate.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _np(a, dtype):
    """Host numpy view (C-contiguous) of an array or a torch tensor."""
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def voxel(p, dims, scale: float = 1.0) -> int:
    """Linear voxel index lin = x + X*(y + Y*z) of one point, or -1 (no voxel)."""
    d = np.asarray(dims, dtype=np.int32)
    p = np.asarray(p, dtype=np.float32)
    return int(_load().oracle_voxel(float(p[0]), float(p[1]), float(p[2]),
                                    float(np.float32(scale)), _ptr(d)))


# the counting modes of the library (same numbering as its mode option)
MODE_PASSTHROUGH, MODE_END, MODE_BOTH_ENDS, MODE_SEED_END = 0, 1, 2, 3


def count(points, offsets, roi, lab, N: int, M: int, scale: float = 1.0, mode: int = MODE_PASSTHROUGH,
          upsample: int = 1) -> np.ndarray:
    """C[N, M] (int64).

    points [P,3] float32, offsets [S+1] int64, roi/lab [Z,Y,X] int32.
    mode 0: pass-through (rows and labels passed through, oracle_count);
    mode 1: rows passed through x label of the last point (oracle_count_endpoint);
    mode 2: rows passed through x labels of the first and last points;
    mode 3: one count per streamline at (row of its first point, label of its last point)
            (oracle_count_seed_endpoint).
    upsample u > 1 (pass-through only): u - 1 evenly spaced points inserted between neighbouring
            points before counting (oracle_count_upsampled).
    """
    pts = _np(points, np.float32).reshape(-1, 3)
    off = _np(offsets, np.int64).reshape(-1)
    roi = _np(roi, np.int32)
    lab = _np(lab, np.int32)
    if roi.shape != lab.shape or roi.ndim != 3:
        raise ValueError("roi and lab must be [Z,Y,X] volumes of one shape")
    S = off.shape[0] - 1
    if S < 0 or off[0] != 0 or off[-1] != pts.shape[0] or np.any(np.diff(off) < 0):
        raise ValueError("offsets must start at 0, be nondecreasing and end at P")
    dims = np.array(roi.shape[::-1], dtype=np.int32)
    C = np.zeros((N, M), dtype=np.int64)
    lib = _load()
    args = (_ptr(pts), _ptr(off), S, _ptr(roi), _ptr(lab), _ptr(dims), int(N), int(M), float(np.float32(scale)))
    if upsample != 1:
        if mode != MODE_PASSTHROUGH or upsample < 1:
            raise ValueError("upsampling is defined for the pass-through mode, u >= 1")
        rc = lib.oracle_count_upsampled(*args, int(upsample), _ptr(C))
    elif mode == MODE_PASSTHROUGH:
        rc = lib.oracle_count(*args, _ptr(C))
    elif mode in (MODE_END, MODE_BOTH_ENDS):
        rc = lib.oracle_count_endpoint(*args, 1 if mode == MODE_BOTH_ENDS else 0, _ptr(C))
    elif mode == MODE_SEED_END:
        rc = lib.oracle_count_seed_endpoint(*args, _ptr(C))
    else:
        raise ValueError(f"unknown mode {mode}")
    if rc != 0:
        raise RuntimeError(f"oracle count (mode {mode}) failed ({rc})")
    return C


def count_chunked(points, offsets, roi, lab, N: int, M: int, scale: float = 1.0,
                  streamlines_per_chunk: int = 1 << 18, workers: int = 1, mode: int = MODE_PASSTHROUGH,
                  upsample: int = 1) -> np.ndarray:
    """The same matrix, computed as a sum of ``count`` over streamline ranges.

    C is a sum over streamlines, so it is additive over any split of the
    streamline list (Section 2 "Method": every streamline adds its own pairs).
    The split only bounds host memory and lets a large workload use several
    processes; each range goes through the unchanged oracle.
    """
    off = _np(offsets, np.int64).reshape(-1)
    S = off.shape[0] - 1
    bounds = list(range(0, S, streamlines_per_chunk)) + [S]
    pts = points
    if hasattr(pts, "detach"):
        pts = pts.detach()
    C = np.zeros((N, M), dtype=np.int64)
    jobs = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        pa, pb = int(off[a]), int(off[b])
        jobs.append((pts[pa:pb], off[a:b + 1] - off[a]))
    if workers <= 1:
        for p, o in jobs:
            C += count(p, o, roi, lab, N, M, scale, mode, upsample)
        return C
    import concurrent.futures as cf
    roi_np, lab_np = _np(roi, np.int32), _np(lab, np.int32)
    # ctypes releases the GIL during the call, so threads run the C oracle in parallel.
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        futs = [ex.submit(count, _np(p, np.float32), o, roi_np, lab_np, N, M, scale, mode, upsample)
                for p, o in jobs]
        for f in futs:
            C += f.result()
    return C


def parcellate(C):
    """(label [N] int32, frac [N, M] float32, sums [N] int64) of a connectivity matrix (oracle_parcellate):
    label = lowest argmax of each row or -1 without a positive entry; frac = row fractions taken in
    double and rounded to float (0 for a row whose sum is not positive)."""
    C = _np(C, np.int64)
    N, M = C.shape
    label = np.zeros(N, np.int32)
    frac = np.zeros((N, M), np.float32)
    sums = np.zeros(N, np.int64)
    rc = _load().oracle_parcellate(_ptr(C), int(N), int(M), _ptr(label), _ptr(frac), _ptr(sums))
    if rc != 0:
        raise RuntimeError(f"oracle_parcellate failed ({rc})")
    return label, frac, sums
