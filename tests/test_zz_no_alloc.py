"""GPU test of fastcod_volume_count_noalloc, the counting entry point that allocates nothing: its
scratch lives in the library's fixed device area.  Two calls in a row through the C-ABI, the
second with a smaller input, each equal to fastcod_volume_count on the same inputs (and the small
one to the oracle); device memory is unchanged across a call."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth

pytestmark = pytest.mark.gpu


def _free_bytes():
    hip = ctypes.CDLL("libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def _noalloc(fc, vol, points, offsets, C, opts=None):
    lib = fc.load()
    f = lib.fastcod_volume_count_noalloc
    # the signature of include/fastcod.h, set here as well: without it ctypes would pass the 64-bit
    # pointers as 32-bit ints
    vp = ctypes.c_void_p
    f.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.POINTER(fc.Opts), vp]
    f.restype = ctypes.c_int
    o = opts if opts is not None else lib.fastcod_default_opts()
    st = torch.cuda.current_stream().cuda_stream
    return f(vol.handle, points.data_ptr(), offsets.data_ptr(), int(offsets.shape[0]) - 1, C.data_ptr(),
             ctypes.byref(o), st)


def test_noalloc_matches_volume_count_two_calls(fc):
    vols = synth.volumes_125mm()
    big = synth.make_125mm(seed=31, S=(1 << 21), device="cuda", vols=vols)     # the largest call it takes
    small = synth.make_125mm(seed=32, S=20_000, device="cuda", vols=vols)
    vol = fc.Volume(big.roi, big.lab, big.N, big.M)
    ref_big = vol.count(big.points, big.offsets)
    ref_small = vol.count(small.points, small.offsets)
    C1 = torch.full((big.N, big.M), -9, dtype=torch.int32, device="cuda")
    C2 = torch.full((big.N, big.M), -9, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    print(f"noalloc: big S={big.S} P={big.P}, small S={small.S} P={small.P}", flush=True)
    assert _noalloc(fc, vol, big.points, big.offsets, C1) == fc.OK, fc.load().fastcod_last_error()
    torch.cuda.synchronize()
    free0 = _free_bytes()
    assert _noalloc(fc, vol, small.points, small.offsets, C2) == fc.OK, fc.load().fastcod_last_error()
    torch.cuda.synchronize()
    assert _free_bytes() == free0          # the second call took no device memory
    assert torch.equal(C1, ref_big)
    assert torch.equal(C2, ref_small)
    exp = oracle.count(small.points, small.offsets, small.roi, small.lab, small.N, small.M)
    assert exp.sum() > 0
    np.testing.assert_array_equal(C2.cpu().numpy(), exp)
    vol.close()


@pytest.mark.parametrize("mode,up,acc,scale", [(1, 1, False, 1.0), (2, 1, True, 1.0), (0, 2, False, 1.7857143),
                                               (3, 1, False, 1.0), (0, 1, False, 1.7857143)])
def test_noalloc_options_match_volume_count(fc, mode, up, acc, scale):
    w = synth.make_sr(seed=41, S=60_000, device="cuda") if scale != 1.0 else \
        synth.make_batch_subject(5, S=60_000, device="cuda")
    vol = fc.Volume(w.roi, w.lab, w.N, w.M)
    init = torch.randint(0, 5, (w.N, w.M), dtype=torch.int32, device="cuda") if acc else \
        torch.full((w.N, w.M), -9, dtype=torch.int32, device="cuda")
    ref = vol.count(w.points, w.offsets, scale=scale, upsample=up, mode=mode, accumulate=acc, out=init.clone())
    got = init.clone()
    o = fc.make_opts(scale=scale, upsample=up, accumulate=acc, mode=mode, variant=fc.VARIANT_STREAM)
    torch.cuda.synchronize()
    print(f"noalloc options: mode={mode} up={up} acc={acc} scale={scale} S={w.S}", flush=True)
    assert _noalloc(fc, vol, w.points, w.offsets, got, o) == fc.OK, fc.load().fastcod_last_error()
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert int(ref.sum()) > (int(init.sum()) if acc else 0)
    vol.close()


def test_noalloc_rejects_too_many_streamlines(fc):
    w = synth.make_tiny64(seed=3, S=100, device="cuda")
    vol = fc.Volume(w.roi, w.lab, w.N, w.M)
    off = torch.zeros((1 << 21) + 2, dtype=torch.int64, device="cuda")
    C = torch.zeros((w.N, w.M), dtype=torch.int32, device="cuda")
    assert _noalloc(fc, vol, w.points, off, C) == fc.EINVAL
    vol.close()


def test_noalloc_degenerate_inputs(fc):
    # no streamlines, and only empty streamlines: C is zeroed (and left alone when accumulating)
    w = synth.make_tiny64(seed=5, S=500, device="cuda")
    vol = fc.Volume(w.roi, w.lab, w.N, w.M)
    # (no points at all; the library takes a non-NULL point pointer whenever there are streamlines)
    pts = torch.zeros((1, 3), dtype=torch.float32, device="cuda")
    for n_off in (1, 9):
        off = torch.zeros(n_off, dtype=torch.int64, device="cuda")
        C = torch.full((w.N, w.M), -9, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        print(f"noalloc degenerate: S={n_off - 1}", flush=True)
        assert _noalloc(fc, vol, pts, off, C) == fc.OK, fc.load().fastcod_last_error()
        torch.cuda.synchronize()
        assert not C.any()
        C.fill_(3)
        assert _noalloc(fc, vol, pts, off, C, fc.make_opts(accumulate=True)) == fc.OK, fc.load().fastcod_last_error()
        torch.cuda.synchronize()
        assert bool((C == 3).all())
    vol.close()
