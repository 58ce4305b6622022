"""GPU tests of fastcod_release and the per-stream workspace cache: device memory returns to its
baseline after counting on several streams and releasing; release beside counts running on another
thread neither crashes nor changes any count (it keeps a workspace in use and reports EBUSY)."""
import ctypes
import threading

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


@pytest.fixture(scope="module")
def work():
    w = synth.make_batch_subject(7, S=40_000, device="cuda")
    exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    assert exp.sum() > 0
    return w, exp


def _warm(fc, w, streams):
    """A count on every stream, then a release: the first launch loads the library's code objects
    (and its static device data) and the first use of a stream sets up its hardware queue; both stay
    for the life of the process and are no workspace."""
    C = torch.empty((w.N, w.M), dtype=torch.int32, device="cuda")
    for st in [None] + list(streams):
        fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=st)
        fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, mode=fc.MODE_BOTH_ENDS, stream=st)
    torch.cuda.synchronize()
    fc.release()


def test_release_returns_device_memory(fc, work):
    w, exp = work
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs = [torch.full((w.N, w.M), -1, dtype=torch.int32, device="cuda") for _ in streams]
    _warm(fc, w, streams)
    torch.cuda.synchronize()
    base = _free_bytes()
    for st, C in zip(streams, outs):
        fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=st)
        fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=st, mode=fc.MODE_BOTH_ENDS)
        fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=st)
    torch.cuda.synchronize()
    used = base - _free_bytes()
    print(f"three workspaces hold {used} bytes", flush=True)
    assert used > 0
    for C in outs:
        np.testing.assert_array_equal(C.cpu().numpy(), exp)
    fc.release()
    after = _free_bytes()
    print(f"free before {base}, after release {after} (difference {base - after})", flush=True)
    assert after == base, (base, after)


def test_workspace_cache_is_bounded(fc, work):
    """Counts on twelve streams keep at most eight workspaces on the device."""
    w, exp = work
    C = torch.zeros((w.N, w.M), dtype=torch.int32, device="cuda")
    streams = [torch.cuda.Stream() for _ in range(12)]
    _warm(fc, w, streams)
    torch.cuda.synchronize()
    base = _free_bytes()
    fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=streams[0])
    torch.cuda.synchronize()
    one = base - _free_bytes()
    for st in streams[1:]:
        fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=st)
        st.synchronize()
    torch.cuda.synchronize()
    used = base - _free_bytes()
    print(f"one workspace {one} bytes, twelve streams {used} bytes", flush=True)
    assert used <= 8 * one + (64 << 20)
    np.testing.assert_array_equal(C.cpu().numpy(), exp)
    fc.release()


def test_release_beside_counts_on_another_thread(fc, work):
    w, exp = work
    stop = threading.Event()
    errors, results = [], []

    def counter():
        try:
            st = torch.cuda.Stream()
            C = torch.empty((w.N, w.M), dtype=torch.int32, device="cuda")
            for _ in range(40):
                fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=st)
                st.synchronize()
                results.append(bool(np.array_equal(C.cpu().numpy(), exp)))
        except Exception as e:   # reported below
            errors.append(e)
        finally:
            stop.set()

    th = threading.Thread(target=counter)
    th.start()
    busy = ok = 0
    lib = fc.load()
    while not stop.is_set():
        rc = lib.fastcod_release()
        if rc == fc.EBUSY:
            busy += 1
        else:
            assert rc == fc.OK, lib.fastcod_last_error()
            ok += 1
    th.join()
    print(f"release: {ok} ok, {busy} busy; {len(results)} counts", flush=True)
    assert not errors, errors
    assert len(results) == 40 and all(results)
    fc.release()
