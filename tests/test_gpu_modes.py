"""GPU parity of the endpoint modes (fastcod_opts.mode) against the oracle, bit-exact.

mode 1: rows passed through x label of the last point (Alg. 2 as printed); mode 2: x labels of the
first and last points; mode 3: Alg. 1's count, one per streamline at (row of its first point,
label of its last point).  Every kernel variant, the resident-volume path, the set-overflow
fallback, runs of empty streamlines (which share their start with the next streamline), the
super-resolution scale, and the full 1.25 mm and 0.7 mm subjects.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth
from tests import _cases

pytestmark = pytest.mark.gpu

VARIANTS = [0, 1, 2]
MODES = [1, 2, 3]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(fc, w, mode, variant=0, scale=None, **kw):
    C = fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=(w.scale if scale is None else scale),
                 variant=variant, mode=mode, **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy().astype(np.int64)


def _wl(points, offsets, roi, lab, N, M, scale=1.0, name="case"):
    return synth.Workload(name, torch.as_tensor(np.ascontiguousarray(points, np.float32)),
                          torch.as_tensor(np.ascontiguousarray(offsets, np.int64)),
                          torch.as_tensor(np.ascontiguousarray(roi, np.int32)),
                          torch.as_tensor(np.ascontiguousarray(lab, np.int32)), int(N), int(M), scale)


def _expect(w, mode, scale=None):
    return oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=(w.scale if scale is None else scale),
                        mode=mode)


@pytest.mark.parametrize("mode", [0] + MODES)
@pytest.mark.parametrize("variant", VARIANTS)
def test_golden_endpoints(fc, mode, variant):
    g = _cases.load_golden("toy_endpoints.json")
    key = {0: "C_passthrough", 1: "C_end", 2: "C_both_ends", 3: "C_seed_end"}[mode]
    w = _wl(g["points"], g["offsets"], g["roi"], g["lab"], g["N"], g["M"]).to("cuda")
    np.testing.assert_array_equal(_run(fc, w, mode, variant), g[key])


@pytest.mark.parametrize("seed", range(10))
def test_random_small(fc, seed):
    w = synth.random_small(seed, N=(None if seed % 3 else 6), bad_values=(seed % 2 == 0),
                           dims=[(12, 10, 9), (7, 16, 5), (33, 3, 18), (70, 9, 11)][seed % 4], S=150, max_len=300)
    g = w.to("cuda")
    for scale in (1.0, 1.7857143):
        for mode in MODES:
            exp = _expect(w, mode, scale)
            for v in VARIANTS:
                np.testing.assert_array_equal(_run(fc, g, mode, v, scale=scale), exp,
                                              err_msg=f"mode {mode} variant {v} scale {scale}")


def _with_empty_runs(w, seed):
    """The same streamlines with runs of empty ones inserted (1 to 140 long, some longer than a
    64-start block): empty streamlines share their start with the next one."""
    rng = np.random.default_rng(seed)
    off = w.offsets.cpu().numpy()
    new = [0]
    for s in range(len(off) - 1):
        if rng.random() < 0.15:
            new.extend([new[-1]] * int(rng.integers(1, 141)))
        new.append(new[-1] + int(off[s + 1] - off[s]))
    new.extend([new[-1]] * 5)
    return _wl(w.points.cpu().numpy(), np.array(new), w.roi.cpu().numpy(), w.lab.cpu().numpy(), w.N, w.M,
               name="empty-runs")


@pytest.mark.parametrize("mode", [0] + MODES)
def test_runs_of_empty_streamlines(fc, mode):
    w = _with_empty_runs(synth.make_tiny64(seed=8, S=4000), 3)
    exp = _expect(w, mode)
    g = w.to("cuda")
    for v in VARIANTS:
        np.testing.assert_array_equal(_run(fc, g, mode, v), exp, err_msg=f"variant {v}")


@pytest.mark.parametrize("mode", MODES)
def test_tiny64_full_and_resident_volume(fc, mode):
    w = synth.make_tiny64(seed=2, S=10_000, device="cuda")
    exp = _expect(w, mode)
    for v in VARIANTS:
        np.testing.assert_array_equal(_run(fc, w, mode, v), exp, err_msg=f"variant {v}")
    vol = fc.Volume(w.roi, w.lab, w.N, w.M)
    got = vol.count(w.points, w.offsets, mode=mode)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), exp)
    # accumulate adds the same matrix again
    vol.count(w.points, w.offsets, mode=mode, accumulate=True, out=got)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), 2 * exp)
    vol.close()


def _overflow_case():
    rng = np.random.default_rng(17)
    X, Y, Z = 300, 40, 30
    roi = np.arange(X * Y * Z, dtype=np.int32).reshape(Z, Y, X)
    lab = rng.integers(-1, 40, size=(Z, Y, X)).astype(np.int32)
    parts, off = [], [0]
    for _ in range(200):
        T = int(rng.integers(1, 1500))
        o = np.array([rng.uniform(0, X), rng.uniform(0, Y), rng.uniform(0, Z)])
        d = rng.normal(size=3)
        d[0] = abs(d[0]) * 4
        d /= np.linalg.norm(d)
        parts.append((o + np.arange(T)[:, None] * 0.5 * d).astype(np.float32))
        off.append(off[-1] + T)
    return _wl(np.concatenate(parts), np.array(off), roi, lab, X * Y * Z, 40, name="overflow")


@pytest.mark.parametrize("mode", MODES)
def test_set_overflow_fallback(fc, mode):
    w = _overflow_case()
    exp = _expect(w, mode)
    g = w.to("cuda")
    for v in VARIANTS:
        np.testing.assert_array_equal(_run(fc, g, mode, v), exp, err_msg=f"variant {v}")


def test_bad_mode_rejected(fc):
    w = synth.random_small(1).to("cuda")
    with pytest.raises(fc.FastcodError) as e:
        fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, mode=4)
    assert e.value.status == fc.EINVAL


def _full(fc, w, modes, variants=(0,), workers=16):
    _say(f"[modes] {w.name}: S={w.S} P={w.P} N={w.N} M={w.M} scale={w.scale}")
    got = {}
    for mode in modes:
        exp = oracle.count_chunked(w.points.cpu(), w.offsets.cpu(), w.roi.cpu(), w.lab.cpu(), w.N, w.M,
                                   scale=w.scale, streamlines_per_chunk=1 << 15, workers=workers, mode=mode)
        for v in variants:
            got[mode] = _run(fc, w, mode, v)
            np.testing.assert_array_equal(got[mode], exp, err_msg=f"mode {mode} variant {v}")
        _say(f"[modes] {w.name}: mode {mode} bit-exact ({int(exp.sum())} pairs)")
    return got


def test_125mm_full(fc):
    _full(fc, synth.make_125mm(device="cuda"), MODES, VARIANTS)


def test_sr_job(fc):
    _full(fc, synth.make_sr(S=100_000, device="cuda"), MODES, VARIANTS)


def test_07mm_full_and_orderings(fc):
    w = synth.make_07mm(device="cuda")
    got = _full(fc, w, [1, 3])
    both = _run(fc, w, 2)
    passthrough = _run(fc, w, 0)
    # entrywise: seed-to-end <= end <= both ends <= pass-through
    assert np.all(got[3] <= got[1]) and np.all(got[1] <= both) and np.all(both <= passthrough)
