"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of oracle/oracle.c with one plausible mistake (a dropped term, a
wrong bound, a transposed operand or index, a missing set operation), compiled with gcc
into a temporary library.  The pin battery (golden toy case, rounding facts, closed-form
lines, brute force, scale) must reject every mutant and accept the unmodified source.
Mutants only ever write inside C's N*M entries, so none of them can corrupt memory.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2302_09247_amd import synth
from tests import _cases

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "no_half_offset": ("float t = q + 0.5f;", "float t = q;"),
    "round_half_away": ("float f = floorf(t);", "float f = roundf(q);"),
    "upper_bound_inclusive": ("!((double)f < (double)dims[k])", "!((double)f <= (double)dims[k])"),
    "drops_voxel_zero": ("if (!(f >= 0.0f)", "if (!(f > 0.0f)"),
    "transposed_volume_layout": ("return v[0] + (int64_t)dims[0] * (v[1] + (int64_t)dims[1] * v[2]);",
                                 "return v[2] + (int64_t)dims[2] * (v[1] + (int64_t)dims[1] * v[0]);"),
    "no_roi_dedupe": ("nI = sort_unique(I, nI);", "(void)0;"),
    "no_label_dedupe": ("nL = sort_unique(L, nL);", "(void)0;"),
    "transposed_C": ("C[(int64_t)I[x] * M + L[y]] += 1;", "C[(int64_t)L[y] * N + I[x]] += 1;"),
    "skips_last_point": ("for (int64_t j = a; j < b; ++j) {", "for (int64_t j = a; j < b - 1; ++j) {"),
    "endpoint_label_only": ("if (m >= 0 && m < M)\n                L[nL++] = m;",
                            "if (m >= 0 && m < M && j == b - 1)\n                L[nL++] = m;"),
    "drops_row_zero": ("if (r >= 0 && r < N)", "if (r > 0 && r < N)"),
    "first_label_only": ("for (int64_t y = 0; y < nL; ++y)", "for (int64_t y = 0; y < nL && y < 1; ++y)"),
    "ignores_scale": ("float q = p[k] * scale;", "float q = p[k];"),
    "uses_x_bound_everywhere": ("!((double)f < (double)dims[k])", "!((double)f < (double)dims[0])"),
    # endpoint modes (oracle_count_endpoint, oracle_count_seed_endpoint)
    "end_label_from_first_point": ("int32_t e_last = label_at(points + 3 * (b - 1),",
                                   "int32_t e_last = label_at(points + 3 * a,"),
    "shared_end_label_counted_twice": ("if (e_first == e_last)\n            e_first = -1;",
                                       "if (0)\n            e_first = -1;"),
    "end_mode_no_row_dedupe": ("nI = sort_unique(I, nI);\n        for (int64_t x = 0; x < nI; ++x) {\n            if (e_last",
                               "(void)0;\n        for (int64_t x = 0; x < nI; ++x) {\n            if (e_last"),
    "end_mode_skips_first_point_rows": ("for (int64_t j = a; j < b; ++j) {\n            int32_t r = row_at(",
                                        "for (int64_t j = a + 1; j < b; ++j) {\n            int32_t r = row_at("),
    "seed_row_from_last_point": ("int32_t seed_row = row_at(points + 3 * a,",
                                 "int32_t seed_row = row_at(points + 3 * (b - 1),"),
    "seed_end_label_from_first_point": ("int32_t end_label = label_at(points + 3 * (b - 1),",
                                        "int32_t end_label = label_at(points + 3 * a,"),
    "label_at_drops_label_zero": ("return (lab[lin] >= 0 && lab[lin] < M) ? lab[lin] : -1;",
                                  "return (lab[lin] > 0 && lab[lin] < M) ? lab[lin] : -1;"),
    "row_at_drops_row_zero": ("return (roi[lin] >= 0 && roi[lin] < N) ? roi[lin] : -1;",
                              "return (roi[lin] > 0 && roi[lin] < N) ? roi[lin] : -1;"),
    # parcellation outputs (oracle_parcellate)
    "argmax_highest_on_tie": ("(best < 0 || row[m] > row[best])", "(best < 0 || row[m] >= row[best])"),
    "empty_row_gets_label_zero": ("if (row[m] > 0 && (best < 0 ||", "if ((best < 0 ||"),
    "fraction_in_float": ("(float)((double)row[m] / (double)total)", "((float)row[m] / (float)total)"),
    "fraction_over_M": ("(float)((double)row[m] / (double)total)", "(float)((double)row[m] / (double)M)"),
    "row_sum_skips_last": ("for (int32_t m = 0; m < M; ++m) {\n            total += row[m];",
                           "for (int32_t m = 0; m < M - 1; ++m) {\n            total += row[m];"),
    # upsampling (oracle_count_upsampled)
    "upsample_wrong_spacing": ("float at = (float)t / (float)u;", "float at = (float)t / (float)(u + 1);"),
    "upsample_inserts_nothing": ("for (int32_t t = 1; t < u; ++t) {", "for (int32_t t = 1; t < 1; ++t) {"),
    "upsample_unscaled_neighbours": ("float qk = points[3 * j + k] * scale;\n                    float qn = points[3 * (j + 1) + k] * scale;",
                                     "float qk = points[3 * j + k];\n                    float qn = points[3 * (j + 1) + k];"),
    "upsample_drops_last_point": ("D[3 * n + k] = points[3 * j + k] * scale;              /* q_j */\n            ++n;\n            if (j + 1 == b)\n                break;",
                                  "D[3 * n + k] = points[3 * j + k] * scale;              /* q_j */\n            if (j + 1 == b)\n                break;\n            ++n;"),
}


def _build(src_text, tmp_path, name):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src_text)
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c), "-lm"])
    lib = ctypes.CDLL(str(so))
    lib.oracle_voxel.restype = ctypes.c_int64
    lib.oracle_voxel.argtypes = [ctypes.c_float] * 4 + [ctypes.c_void_p]
    lib.oracle_count.restype = ctypes.c_int
    common = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
              ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float]
    lib.oracle_count.argtypes = common + [ctypes.c_void_p]
    lib.oracle_count_endpoint.restype = ctypes.c_int
    lib.oracle_count_endpoint.argtypes = common + [ctypes.c_int, ctypes.c_void_p]
    lib.oracle_count_seed_endpoint.restype = ctypes.c_int
    lib.oracle_count_seed_endpoint.argtypes = common + [ctypes.c_void_p]
    lib.oracle_parcellate.restype = ctypes.c_int
    lib.oracle_parcellate.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_count_upsampled.restype = ctypes.c_int
    lib.oracle_count_upsampled.argtypes = common + [ctypes.c_int32, ctypes.c_void_p]
    return lib


def _count(lib, points, offsets, roi, lab, N, M, scale=1.0, mode=0):
    p = np.ascontiguousarray(points, np.float32)
    o = np.ascontiguousarray(offsets, np.int64)
    r = np.ascontiguousarray(roi, np.int32)
    lb = np.ascontiguousarray(lab, np.int32)
    d = np.array(r.shape[::-1], np.int32)
    C = np.zeros((N, M), np.int64)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)   # noqa: E731
    args = (ptr(p), ptr(o), o.shape[0] - 1, ptr(r), ptr(lb), ptr(d), N, M, float(np.float32(scale)))
    if mode == 0:
        rc = lib.oracle_count(*args, ptr(C))
    elif mode in (1, 2):
        rc = lib.oracle_count_endpoint(*args, mode - 1, ptr(C))
    elif mode >= 10:   # upsampled pass-through, u = mode - 10
        rc = lib.oracle_count_upsampled(*args, mode - 10, ptr(C))
    else:
        rc = lib.oracle_count_seed_endpoint(*args, ptr(C))
    assert rc == 0
    return C


def _battery(lib):
    """Names of the failed pins (empty = every pin passed)."""
    failed = []
    g = _cases.load_golden("toy_two_streamlines.json")
    if not np.array_equal(_count(lib, g["points"], g["offsets"], g["roi"], g["lab"], g["N"], g["M"]), g["C"]):
        failed.append("golden")
    for value, X, exp in _cases.ROUNDING_PINS:
        for axis in range(3):
            dims = [3, 3, 3]
            dims[axis] = X
            p = [1.0, 1.0, 1.0]
            p[axis] = value
            v = [1, 1, 1]
            v[axis] = exp
            want = -1 if exp < 0 else v[0] + dims[0] * (v[1] + dims[1] * v[2])
            d = np.array(dims, np.int32)
            if lib.oracle_voxel(*[float(np.float32(c)) for c in p], 1.0, d.ctypes.data_as(ctypes.c_void_p)) != want:
                failed.append(f"rounding {value}")
    lab_of = lambda M: (lambda x, y, z: ((x + 2 * y + 3 * z) % (M + 1)) - 1)   # noqa: E731
    for origin, step, T, dims, M in [((0.25, 2.0, 1.0), (0.5, 0.0, 0.0), 23, (13, 4, 3), 4),
                                     ((0.125, 0.375, 0.0625), (0.25, 0.25, 0.25), 40, (11, 12, 13), 6)]:
        pts, off, roi, lab, N, M, Cexp = _cases.line_case(origin, step, T, dims, M, lab_of(M))
        if not np.array_equal(_count(lib, pts, off, roi, lab, N, M), Cexp):
            failed.append(f"line {origin}")
    for seed in range(4):
        w = synth.random_small(seed, N=(None if seed % 2 else 6), bad_values=True)
        args = (w.points.numpy(), w.offsets.numpy(), w.roi.numpy(), w.lab.numpy(), w.N, w.M)
        for scale in (1.0, 1.7857143):
            if not np.array_equal(_count(lib, *args, scale=scale), brute.brute_count(*args, scale=scale)):
                failed.append(f"brute {seed} {scale}")
    # endpoint modes: the hand-worked case and the dense brute force
    g = _cases.load_golden("toy_endpoints.json")
    for mode, key in ((1, "C_end"), (2, "C_both_ends"), (3, "C_seed_end")):
        if not np.array_equal(_count(lib, g["points"], g["offsets"], g["roi"], g["lab"], g["N"], g["M"], mode=mode),
                              g[key]):
            failed.append(f"golden endpoints mode {mode}")
        for seed in range(4):
            w = synth.random_small(seed, N=(None if seed % 2 else 6), bad_values=True)
            args = (w.points.numpy(), w.offsets.numpy(), w.roi.numpy(), w.lab.numpy(), w.N, w.M)
            if not np.array_equal(_count(lib, *args, mode=mode), brute.brute_count_ends(*args, mode=mode)):
                failed.append(f"brute ends {seed} mode {mode}")
    failed += _battery_parcellate(lib)
    # upsampling: the hand-worked case and the numpy densification
    g = _cases.load_golden("toy_upsample.json")
    for u in (2, 3, 4):
        if not np.array_equal(_count(lib, g["points"], g["offsets"], g["roi"], g["lab"], g["N"], g["M"], mode=10 + u),
                              g[f"C_u{u}"]):
            failed.append(f"golden upsample {u}")
    for seed in range(3):
        w = synth.random_small(seed, N=(None if seed % 2 else 6), bad_values=True)
        pts, off = brute.brute_upsample(w.points.numpy(), w.offsets.numpy(), 1.7857143, 3)
        want = brute.brute_count(pts, off, w.roi.numpy(), w.lab.numpy(), w.N, w.M)
        args = (w.points.numpy(), w.offsets.numpy(), w.roi.numpy(), w.lab.numpy(), w.N, w.M)
        if not np.array_equal(_count(lib, *args, scale=1.7857143, mode=13), want):
            failed.append(f"brute upsample {seed}")
    return failed


def _battery_parcellate(lib):
    """Hand-worked rows and exact-rational fractions (counts up to 2^26)."""
    from tests import test_oracle_parcellate as tp
    failed = []
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)   # noqa: E731

    def run(C):
        C = np.ascontiguousarray(C, np.int64)
        N, M = C.shape
        lab, frac, sums = np.zeros(N, np.int32), np.zeros((N, M), np.float32), np.zeros(N, np.int64)
        assert lib.oracle_parcellate(ptr(C), N, M, ptr(lab), ptr(frac), ptr(sums)) == 0
        return lab, frac, sums

    import json
    from fractions import Fraction
    g = json.load(open(tp.GOLDEN))
    lab, frac, sums = run(np.array(g["C"]))
    if not (np.array_equal(lab, g["labels"]) and np.array_equal(sums, g["sums"])):
        failed.append("parcellation golden labels/sums")
    for i, row in enumerate(g["fractions"]):
        if not all(tp._close_to_rational(frac[i, m], Fraction(t)) for m, t in enumerate(row)):
            failed.append(f"parcellation golden fractions row {i}")
    rng = np.random.default_rng(3)
    C = rng.integers(1 << 24, 1 << 26, size=(8, 5)).astype(np.int64)
    lab, frac, sums = run(C)
    for i in range(C.shape[0]):
        s = int(C[i].sum())
        if sums[i] != s or not all(tp._close_to_rational(frac[i, m], Fraction(int(C[i, m]), s)) for m in range(5)):
            failed.append(f"parcellation large counts row {i}")
            break
    return failed


def test_unmodified_oracle_passes_battery(tmp_path):
    assert _battery(_build(open(SRC).read(), tmp_path, "orig")) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found in oracle.c"
    failed = _battery(_build(src.replace(old, new, 1), tmp_path, name))
    assert failed, f"planted mistake {name} was not caught by any pin"
