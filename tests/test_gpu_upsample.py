"""GPU parity of the upsampled pass-through count (fastcod_opts.upsample = u) with the oracle,
bit-exact: every variant (flat stream, wave, auto), u = 2, 3, 4, the super-resolution scale, runs
of empty streamlines, the set-overflow fallback, a 1.25 mm -> 0.7 mm super-resolution job in full
and the 1.25 mm subject in full."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth
from tests import _cases
from tests.test_gpu_modes import _overflow_case, _with_empty_runs

pytestmark = pytest.mark.gpu

VARIANTS = [0, 1, 2]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(fc, w, u, variant=0, scale=None):
    C = fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=(w.scale if scale is None else scale),
                 variant=variant, upsample=u)
    torch.cuda.synchronize()
    return C.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("u", [1, 2, 3, 4])
@pytest.mark.parametrize("variant", VARIANTS)
def test_golden(fc, u, variant):
    g = _cases.load_golden("toy_upsample.json")
    w = synth.Workload("g", torch.from_numpy(g["points"]), torch.from_numpy(g["offsets"]), torch.from_numpy(g["roi"]),
                       torch.from_numpy(g["lab"]), g["N"], g["M"]).to("cuda")
    np.testing.assert_array_equal(_run(fc, w, u, variant), g[f"C_u{u}"])


@pytest.mark.parametrize("seed", range(8))
def test_random_small(fc, seed):
    w = synth.random_small(seed, N=(None if seed % 3 else 6), bad_values=(seed % 2 == 0),
                           dims=[(12, 10, 9), (7, 16, 5), (33, 3, 18), (70, 9, 11)][seed % 4], S=150, max_len=300)
    g = w.to("cuda")
    for scale in (1.0, 1.7857143):
        for u in (2, 3, 4):
            exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=scale, upsample=u)
            for v in VARIANTS:
                np.testing.assert_array_equal(_run(fc, g, u, v, scale=scale), exp,
                                              err_msg=f"u {u} variant {v} scale {scale}")


@pytest.mark.parametrize("u", [2, 4])
def test_tiny64_and_empty_runs(fc, u):
    w = synth.make_tiny64(seed=4, S=6000)
    for ww in (w, _with_empty_runs(synth.make_tiny64(seed=9, S=3000), 5)):
        exp = oracle.count(ww.points, ww.offsets, ww.roi, ww.lab, ww.N, ww.M, upsample=u, scale=1.25)
        g = ww.to("cuda")
        for v in VARIANTS:
            np.testing.assert_array_equal(_run(fc, g, u, v, scale=1.25), exp, err_msg=f"{ww.name} variant {v}")


@pytest.mark.parametrize("u", [2, 3])
def test_set_overflow_fallback(fc, u):
    w = _overflow_case()
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, upsample=u)
    g = w.to("cuda")
    for v in VARIANTS:
        np.testing.assert_array_equal(_run(fc, g, u, v), exp, err_msg=f"variant {v}")


def test_rejections(fc):
    w = synth.random_small(2).to("cuda")
    for kw in (dict(upsample=5), dict(upsample=0), dict(upsample=2, mode=1)):
        with pytest.raises(fc.FastcodError) as e:
            fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, **kw)
        assert e.value.status == fc.EINVAL


def test_sr_job_upsampled_full(fc):
    # super-resolution as the paper describes it: 1.25 mm streamlines (0.5-voxel steps) scaled by
    # fl32(1.25/0.7) onto the 0.7 mm grid (0.89-voxel spacing), upsampled by 2 to 0.45 voxel
    w = synth.make_sr(S=200_000, device="cuda")
    _say(f"[upsample] sr: S={w.S} P={w.P}")
    exp = oracle.count_chunked(w.points.cpu(), w.offsets.cpu(), w.roi.cpu(), w.lab.cpu(), w.N, w.M, scale=w.scale,
                               streamlines_per_chunk=1 << 14, workers=16, upsample=2)
    for v in VARIANTS:
        np.testing.assert_array_equal(_run(fc, w, 2, v), exp, err_msg=f"variant {v}")
    base = _run(fc, w, 1)
    assert np.all(base <= exp) and exp.sum() > base.sum()


def test_125mm_full_u3(fc):
    w = synth.make_125mm(device="cuda")
    _say(f"[upsample] 1.25mm: S={w.S} P={w.P}")
    exp = oracle.count_chunked(w.points.cpu(), w.offsets.cpu(), w.roi.cpu(), w.lab.cpu(), w.N, w.M,
                               streamlines_per_chunk=1 << 15, workers=16, upsample=3)
    np.testing.assert_array_equal(_run(fc, w, 3), exp)
