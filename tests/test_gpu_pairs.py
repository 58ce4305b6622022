"""GPU parity of the flat-stream path's pair buffer against the oracle, bit-exact.

The flat-stream kernel appends its C updates to per-wavefront slices of `pair_capacity` entries
and adds their histogram into C tile by tile; a full slice sends the rest of its wavefront's
updates to C as atomics.  Capacities from 1 entry (every wavefront overflows at once) to the
default must give the same C, alone, with accumulate, in every mode and with upsampling; a C of
more than 2^26 entries takes the transposed-atomics path instead.  With the default capacity (0),
calls of fewer than 2^17 streamlines on a C of at most 2^20 entries use no pair buffer at all (every
update an atomic into C); an explicit capacity keeps it.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth

pytestmark = pytest.mark.gpu

CAPACITIES = [1, 200, 20_000, 0]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(fc, w, **kw):
    C = fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=w.scale, variant=2, **kw)
    torch.cuda.synchronize()
    return C.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("cap", CAPACITIES)
def test_capacities_tiny64(fc, cap):
    w = synth.make_tiny64(seed=11, S=20_000)
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    g = w.to("cuda")
    np.testing.assert_array_equal(_run(fc, g, pair_capacity=cap), exp)


@pytest.mark.parametrize("seed", range(6))
def test_capacities_random_small(fc, seed):
    w = synth.random_small(seed, dims=[(12, 10, 9), (33, 3, 18), (70, 9, 11)][seed % 3], S=400, max_len=300,
                           bad_values=(seed % 2 == 0))
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    g = w.to("cuda")
    for cap in CAPACITIES:
        np.testing.assert_array_equal(_run(fc, g, pair_capacity=cap), exp, err_msg=f"capacity {cap}")


@pytest.mark.parametrize("cap", [1, 5000, 0])   # (0: no pair buffer for this small call)
def test_accumulate_with_small_slices(fc, cap):
    w = synth.make_tiny64(seed=12, S=8000)
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    g = w.to("cuda")
    base = torch.arange(w.N * w.M, dtype=torch.int32, device="cuda").reshape(w.N, w.M) % 7
    out = base.clone()
    fc.count(g.points, g.offsets, g.roi, g.lab, g.N, g.M, accumulate=True, out=out, variant=2, pair_capacity=cap)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.int64), base.cpu().numpy() + exp)


@pytest.mark.parametrize("mode", [1, 2])
def test_endpoint_modes_with_small_slices(fc, mode):
    w = synth.make_tiny64(seed=13, S=6000)
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, mode=mode)
    g = w.to("cuda")
    for cap in (1, 3000, 0):
        np.testing.assert_array_equal(_run(fc, g, mode=mode, pair_capacity=cap), exp, err_msg=f"capacity {cap}")


@pytest.mark.parametrize("u", [2, 4])
def test_upsampled_with_small_slices(fc, u):
    w = synth.make_tiny64(seed=14, S=4000)
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, upsample=u, scale=1.25)
    g = w.to("cuda")
    for cap in (1, 3000, 0):
        C = fc.count(g.points, g.offsets, g.roi, g.lab, g.N, g.M, scale=1.25, upsample=u, variant=2, pair_capacity=cap)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(C.cpu().numpy().astype(np.int64), exp, err_msg=f"capacity {cap}")


def test_125mm_small_slices(fc):
    # about 2.8 updates per streamline: 2^20 entries over the wavefronts fill many slices
    w = synth.make_125mm(device="cuda")
    _say(f"[pairs] 1.25mm: S={w.S} P={w.P}")
    exp = oracle.count_chunked(w.points.cpu(), w.offsets.cpu(), w.roi.cpu(), w.lab.cpu(), w.N, w.M,
                               streamlines_per_chunk=1 << 15, workers=16)
    for cap in (1 << 20, 0):
        np.testing.assert_array_equal(_run(fc, w, pair_capacity=cap), exp, err_msg=f"capacity {cap}")
    _say(f"[pairs] 1.25mm bit-exact ({int(exp.sum())} updates)")


@pytest.mark.parametrize("S", [(1 << 17) - 1, 1 << 17])
def test_direct_atomics_threshold(fc, S):
    # either side of the streamline count below which a small C skips the pair buffer
    w = synth.make_tiny64(seed=17, S=S)
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    g = w.to("cuda")
    _say(f"[pairs] tiny64 S={S} P={w.P}")
    for cap in (0, 4 * S):
        np.testing.assert_array_equal(_run(fc, g, pair_capacity=cap), exp, err_msg=f"capacity {cap}")


def test_large_C_takes_the_atomic_path(fc):
    # N*M > 2^26: past the histogram's tile table; only the first rows and labels are used
    w = synth.make_tiny64(seed=15, S=3000)
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    g = w.to("cuda")
    N, M = 1 << 13, (1 << 13) + 1
    assert w.N <= N and w.M <= M
    C = fc.count(g.points, g.offsets, g.roi, g.lab, N, M, variant=2)
    torch.cuda.synchronize()
    top = C[: w.N, : w.M].cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(top, exp)
    assert int(C.sum(dtype=torch.int64).item()) == int(exp.sum())
    del C
    torch.cuda.empty_cache()


@pytest.mark.parametrize("batch", [2, 4])
def test_both_batch_sizes(fc, batch):
    # the flat-stream loop's two schedules (64-point windows per pipelined batch), every mode, with
    # upsampling, and with slices small enough to overflow
    w = synth.make_tiny64(seed=16, S=12_000)
    g = w.to("cuda")
    for mode in (0, 1, 2):
        exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, mode=mode)
        for cap in (0, 500):
            np.testing.assert_array_equal(_run(fc, g, mode=mode, batch=batch, pair_capacity=cap), exp,
                                          err_msg=f"mode {mode} capacity {cap}")
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=1.25, upsample=2)
    C = fc.count(g.points, g.offsets, g.roi, g.lab, g.N, g.M, scale=1.25, upsample=2, variant=2, batch=batch)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(C.cpu().numpy().astype(np.int64), exp)
    for seed in range(4):
        s = synth.random_small(seed, dims=[(12, 10, 9), (70, 9, 11)][seed % 2], S=300, max_len=400,
                               bad_values=(seed % 2 == 0))
        exp = oracle.count(s.points, s.offsets, s.roi, s.lab, s.N, s.M)
        np.testing.assert_array_equal(_run(fc, s.to("cuda"), batch=batch), exp, err_msg=f"seed {seed}")
