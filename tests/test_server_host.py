"""Host tests of the request server's scheduling core (csrc/server_core.h), run through a simulated
executor (tests/native/server_sim.cpp, built here with g++): admission against the memory budget,
first-come-first-served order, LRU eviction of idle volumes, chunk coverage, continuous batching,
tick shares (a floor each, the rest oldest first), cancellation, failure, and the threaded
wrapper's wait/timeout.  No GPU, no counting: the counting itself is covered by the GPU tests of the
served form."""
import ctypes
import os
import subprocess
import threading

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD, BEGIN, UPLOAD, TICK, FINAL = range(5)
PENDING, ACTIVE, FINALIZING, DONE = range(4)
OK, EINVAL, ERANGE, ENOMEM, EHIP, EBUSY, ECANCELED, ETIMEDOUT = 0, -1, -2, -3, -4, -5, -6, -7
DEVICE_POINTS, DEVICE_C = 1, 2
KB = 1 << 10
MB = 1 << 20

i32, i64, u32, u64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("sim") / "libserver_sim.so")
    # SERVER_SIM_SANITIZE=1 builds with AddressSanitizer/UBSan (run python with libasan preloaded)
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"] if os.environ.get("SERVER_SIM_SANITIZE") else []
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-Wall", "-Werror", *san,
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2302_09247_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "server_sim.cpp"), "-o", out, "-lpthread"])
    lib = ctypes.CDLL(out)
    lib.arena_new.restype = vp
    lib.arena_new.argtypes = [u64]
    lib.arena_alloc.restype = i64
    lib.arena_alloc.argtypes = [vp, u64]
    lib.arena_free.argtypes = [vp, i64]
    lib.arena_used.restype = u64
    lib.arena_used.argtypes = [vp]
    lib.arena_largest.restype = u64
    lib.arena_largest.argtypes = [vp]
    lib.arena_free_blocks.restype = i64
    lib.arena_free_blocks.argtypes = [vp]
    lib.arena_delete.argtypes = [vp]
    lib.sim_create.restype = vp
    lib.sim_create.argtypes = [u64, i64, i64, i64, i32, i32, i32]
    lib.sim_destroy.argtypes = [vp]
    lib.sim_add_volume.argtypes = [vp, i32, i32, u64, u64, ctypes.POINTER(i32)]
    lib.sim_submit.argtypes = [vp, i32, u32, vp, i64, ctypes.POINTER(u64)]
    lib.sim_step.argtypes = [vp]
    lib.sim_complete.argtypes = [vp, ctypes.c_int]
    lib.sim_auto.argtypes = [vp, ctypes.c_int]
    lib.sim_fail_issue.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.sim_fail_done.argtypes = [vp, ctypes.c_int]
    lib.sim_cancel.argtypes = [vp, u64]
    lib.sim_stop.argtypes = [vp]
    lib.sim_idle.argtypes = [vp]
    lib.sim_state.argtypes = [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.sim_chunks.restype = i64
    lib.sim_chunks.argtypes = [vp, vp, i64]
    lib.sim_ops.restype = i64
    lib.sim_ops.argtypes = [vp, vp, i64]
    lib.sim_stats.argtypes = [vp, vp]
    lib.svc_create.restype = vp
    lib.svc_create.argtypes = [u64, i64, i64, i32, i32]
    lib.svc_add_volume.argtypes = [vp, i32, i32, u64, ctypes.POINTER(i32)]
    lib.svc_submit.argtypes = [vp, i32, vp, i64, ctypes.POINTER(u64)]
    lib.svc_wait.argtypes = [vp, u64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.svc_cancel.argtypes = [vp, u64]
    lib.svc_destroy.argtypes = [vp]
    return lib


class Core:
    """Python view of one simulated core."""

    def __init__(self, lib, budget=64 * MB, tick_points=1000, tick_streamlines=1 << 20, chunk_points=100,
                 max_active=64, upload_window=8, ticks_in_flight=2):
        self.lib = lib
        self.h = lib.sim_create(budget, tick_points, tick_streamlines, chunk_points, max_active, upload_window,
                                ticks_in_flight)
        self.offsets = {}

    def close(self):
        if self.h:
            self.lib.sim_destroy(self.h)
        self.h = None

    def add_volume(self, N=10, M=4, nbytes=MB, tmp=MB):
        vid = i32()
        rc = self.lib.sim_add_volume(self.h, N, M, nbytes, tmp, ctypes.byref(vid))
        return rc, vid.value

    def submit(self, vol, lengths=None, flags=0, offsets=None):
        if offsets is None:
            offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        rid = u64()
        rc = self.lib.sim_submit(self.h, vol, flags, offsets.ctypes.data, len(offsets) - 1, ctypes.byref(rid))
        if rc == OK:
            self.offsets[rid.value] = offsets   # kept alive: the core reads them until done
        return rc, rid.value

    def step(self, complete=None):
        p = self.lib.sim_step(self.h)
        if complete is not None:
            self.lib.sim_complete(self.h, complete)
        return p

    def run(self, limit=10000):
        """Steps, completing every issued operation, until the core is idle."""
        for _ in range(limit):
            self.lib.sim_step(self.h)
            self.lib.sim_complete(self.h, -1)
            if self.lib.sim_idle(self.h):
                self.lib.sim_step(self.h)
                return
        raise AssertionError("core did not become idle")

    def state(self, rid):
        s, st, ch = i32(), i32(), i64()
        if self.lib.sim_state(self.h, rid, ctypes.byref(s), ctypes.byref(st), ctypes.byref(ch)) != 0:
            return None
        return s.value, st.value, ch.value

    def chunks(self):
        n = self.lib.sim_chunks(self.h, None, 0)
        buf = np.zeros(n, dtype=np.int64)
        self.lib.sim_chunks(self.h, buf.ctypes.data, n)
        assert -999 not in buf, "a chunk reached past the uploaded streamlines or skipped some"
        return buf.reshape(-1, 4)   # (tick, req, s0, s1)

    def ops(self):
        n = self.lib.sim_ops(self.h, None, 0)
        buf = np.zeros(5 * max(n, 1), dtype=np.int64)
        self.lib.sim_ops(self.h, buf.ctypes.data, n)
        return buf[:5 * n].reshape(-1, 5)

    def stats(self):
        buf = np.zeros(11, dtype=np.int64)
        self.lib.sim_stats(self.h, buf.ctypes.data)
        keys = ("used", "size", "pending", "active", "completed", "ticks", "builds", "evictions", "failed",
                "largest_free", "live_tokens")
        return dict(zip(keys, buf.tolist()))


@pytest.fixture
def core(sim):
    cores = []

    def make(**kw):
        c = Core(sim, **kw)
        cores.append(c)
        return c
    yield make
    for c in cores:
        c.close()


def _rup(b):
    return (max(b, 1) + 255) // 256 * 256


# ---------------------------------------------------------------------------------------------
def test_arena_random_alloc_free(sim):
    rng = np.random.default_rng(0)
    size = 1 << 24
    a = sim.arena_new(size)
    live = {}
    for it in range(4000):
        if live and (rng.random() < 0.45 or len(live) > 60):
            off = list(live)[rng.integers(len(live))]
            sim.arena_free(a, off)
            del live[off]
        else:
            n = int(rng.integers(1, 1 << 19))
            off = sim.arena_alloc(a, n)
            if off < 0:
                assert sim.arena_largest(a) < _rup(n)
                continue
            assert off % 256 == 0
            for o, m in live.items():   # no overlap with any live block
                assert off + _rup(n) <= o or o + m <= off
            live[off] = _rup(n)
        assert sim.arena_used(a) == sum(live.values())
    for off in list(live):
        sim.arena_free(a, off)
    assert sim.arena_used(a) == 0 and sim.arena_largest(a) == size and sim.arena_free_blocks(a) == 1
    sim.arena_free(a, 12345)   # unknown offsets are ignored
    assert sim.arena_used(a) == 0
    sim.arena_delete(a)


def test_every_streamline_counted_once_per_request(core):
    rng = np.random.default_rng(1)
    c = core(tick_points=5000, chunk_points=300, max_active=5, upload_window=3)
    _, v0 = c.add_volume()
    _, v1 = c.add_volume()
    reqs = {}
    for k in range(12):
        S = int(rng.integers(0, 400))
        lengths = rng.integers(0, 60, size=S)
        lengths[rng.random(S) < 0.1] = 0   # empty streamlines in the mix
        flags = DEVICE_POINTS if k % 3 == 0 else 0
        rc, rid = c.submit(v0 if k % 2 else v1, lengths, flags=flags)
        assert rc == OK
        reqs[rid] = S
    c.run()
    ch = c.chunks()
    for rid, S in reqs.items():
        st = c.state(rid)
        assert st[0] == DONE and st[1] == OK
        mine = ch[ch[:, 1] == rid]
        if S == 0:
            assert len(mine) == 0
            continue
        s0, s1 = mine[:, 2], mine[:, 3]
        assert s0[0] == 0 and s1[-1] == S and np.all(s0[1:] == s1[:-1]) and np.all(s1 > s0)
        assert np.all(np.diff(mine[:, 0]) > 0)   # at most one range of a request per launch
    s = c.stats()
    assert s["active"] == 0 and s["pending"] == 0 and s["completed"] == len(reqs)
    assert s["used"] == 2 * _rup(1 * MB)       # only the two resident volumes remain
    assert s["live_tokens"] == 0


def test_result_copy_after_last_launch(core):
    c = core(tick_points=100, chunk_points=50)
    _, v = c.add_volume()
    _, rid = c.submit(v, [10] * 40)
    c.run()
    ops = c.ops()
    last_tick = max(i for i, o in enumerate(ops) if o[0] == TICK)
    final = [i for i, o in enumerate(ops) if o[0] == FINAL and o[1] == rid]
    assert len(final) == 1 and final[0] > last_tick
    begin = [i for i, o in enumerate(ops) if o[0] == BEGIN and o[1] == rid]
    first_tick = min(i for i, o in enumerate(ops) if o[0] == TICK)
    assert begin[0] < first_tick


def test_new_request_joins_next_launch(core):
    c = core(tick_points=200, chunk_points=50, ticks_in_flight=1)
    _, v = c.add_volume()
    _, a = c.submit(v, [10] * 1000, flags=DEVICE_POINTS)
    for _ in range(3):
        c.step(complete=-1)
    _, b = c.submit(v, [10] * 30, flags=DEVICE_POINTS)
    ticks_before = c.stats()["ticks"]
    c.step(complete=-1)   # admits b
    c.step(complete=-1)
    ch = c.chunks()
    first_b = ch[ch[:, 1] == b][0, 0]
    assert first_b <= ticks_before + 2
    assert c.state(a)[0] != DONE   # b started while a was still running
    c.run()
    assert c.state(a)[:2] == (DONE, OK) and c.state(b)[:2] == (DONE, OK)


def test_tick_shares_floor_then_oldest_first(core):
    # every ready request gets chunk_points of a tick; the rest of the tick goes to the oldest
    c = core(tick_points=1000, chunk_points=100, ticks_in_flight=1)
    _, v = c.add_volume()
    _, a = c.submit(v, [10] * 5000, flags=DEVICE_POINTS)
    _, b = c.submit(v, [10] * 5000, flags=DEVICE_POINTS)
    for _ in range(12):
        c.step(complete=-1)
    ch = c.chunks()
    both = 0
    for t in np.unique(ch[:, 0]):
        sel = ch[ch[:, 0] == t]
        if len(sel) == 2:
            both += 1
            pts = {int(r): int(s1 - s0) * 10 for _, r, s0, s1 in sel}
            assert pts[a] == 900 and pts[b] == 100
    assert both >= 3
    c.run()
    ch = c.chunks()
    last = {r: int(ch[ch[:, 1] == r][:, 0].max()) for r in (a, b)}
    assert last[a] < last[b]   # the older request finished first
    assert c.state(a)[:2] == (DONE, OK) and c.state(b)[:2] == (DONE, OK)


def test_tick_shares_many_requests(core):
    # more ready requests than tick_points / chunk_points: equal parts of the tick, nobody left out
    c = core(tick_points=1000, chunk_points=100, ticks_in_flight=1)
    _, v = c.add_volume()
    ids = [c.submit(v, [1] * 3000, flags=DEVICE_POINTS)[1] for _ in range(20)]
    for _ in range(6):
        c.step(complete=-1)
    ch = c.chunks()
    t = int(ch[:, 0].max())
    sel = ch[ch[:, 0] == t]
    assert sorted(int(r) for r in sel[:, 1]) == sorted(ids)
    assert np.all((sel[:, 3] - sel[:, 2]) == 50)
    c.run()
    assert all(c.state(r)[:2] == (DONE, OK) for r in ids)


def test_finalizing_request_makes_room(core):
    # max_active bounds the requests still counting: one whose result is being copied out lets the
    # next one in
    c = core(tick_points=1000, chunk_points=100, max_active=1)
    _, v = c.add_volume()
    _, a = c.submit(v, [10] * 20, flags=DEVICE_POINTS)
    _, b = c.submit(v, [10] * 20, flags=DEVICE_POINTS)
    for _ in range(8):   # every operation completes except the result copies
        c.step()
        for kind in (BUILD, BEGIN, UPLOAD, TICK):
            c.lib.sim_complete(c.h, kind)
    assert c.state(a)[0] == FINALIZING
    assert c.state(b)[0] in (ACTIVE, FINALIZING)
    c.run()
    assert c.state(a)[:2] == (DONE, OK) and c.state(b)[:2] == (DONE, OK)


def test_tick_streamline_cap(core):
    c = core(tick_points=1 << 30, tick_streamlines=64, chunk_points=1000)
    _, v = c.add_volume()
    _, a = c.submit(v, [1] * 1000, flags=DEVICE_POINTS)
    _, b = c.submit(v, [1] * 1000, flags=DEVICE_POINTS)
    c.run()
    ch = c.chunks()
    for t in np.unique(ch[:, 0]):
        sel = ch[ch[:, 0] == t]
        assert (sel[:, 3] - sel[:, 2]).sum() <= 64


def test_fifo_admission_within_budget(core):
    # volume 1 MB + scratch 1 MB; each request holds about 12 B/point + offsets + C
    c = core(budget=5 * MB, tick_points=1 << 20, chunk_points=1 << 16)
    _, v = c.add_volume(N=100, M=10)
    big = [1000] * 200        # 2.4 MB of points
    rc, a = c.submit(v, big)
    rc2, b = c.submit(v, big)
    rc3, small = c.submit(v, [5] * 10)
    assert rc == rc2 == rc3 == OK
    for _ in range(3):
        c.step()
    assert c.state(a)[0] == ACTIVE
    assert c.state(b)[0] == PENDING
    assert c.state(small)[0] == PENDING   # no overtaking: strictly first come, first served
    c.run()
    for r in (a, b, small):
        assert c.state(r)[:2] == (DONE, OK)


def test_request_that_never_fits_is_refused(core):
    c = core(budget=4 * MB)
    _, v = c.add_volume(N=10, M=4)
    rc, _ = c.submit(v, [100000] * 2)   # 2.4 MB of points + 2 MB of volume and scratch
    assert rc == ENOMEM
    rc, rid = c.submit(v, [100000] * 2, flags=DEVICE_POINTS)   # points already on the device: fits
    assert rc == OK
    c.run()
    assert c.state(rid)[:2] == (DONE, OK)
    rc, _ = c.add_volume(nbytes=3 * MB, tmp=2 * MB)
    assert rc == ENOMEM


def test_lru_eviction_of_idle_volumes(core):
    # two resident volumes (2 MB) leave 1.5 MB: a third build (1 MB + 1 MB scratch) must evict one
    c = core(budget=3 * MB + 512 * KB)
    vols = [c.add_volume(N=8, M=4, nbytes=MB, tmp=MB)[1] for _ in range(3)]
    for vid in vols[:2]:
        _, r = c.submit(vid, [3] * 5, flags=DEVICE_POINTS | DEVICE_C)
        c.run()
        assert c.state(r)[:2] == (DONE, OK)
    s = c.stats()
    assert s["builds"] == 2 and s["evictions"] == 0
    # third volume: 2 MB more needed (1 MB resident + 1 MB scratch) -> evicts the least recently used (vols[0])
    _, r = c.submit(vols[2], [3] * 5, flags=DEVICE_POINTS | DEVICE_C)
    c.run()
    s = c.stats()
    assert s["builds"] == 3 and s["evictions"] == 1
    # vols[1] is still resident (no rebuild); vols[0] is rebuilt
    _, r = c.submit(vols[1], [3] * 5, flags=DEVICE_POINTS | DEVICE_C)
    c.run()
    assert c.stats()["builds"] == 3
    _, r = c.submit(vols[0], [3] * 5, flags=DEVICE_POINTS | DEVICE_C)
    c.run()
    assert c.stats()["builds"] == 4
    ops = c.ops()
    builds = [o[1] for o in ops if o[0] == BUILD]
    assert builds == [vols[0], vols[1], vols[2], vols[0]]


def test_volume_in_use_is_not_evicted(core):
    c = core(budget=3 * MB + 512 * KB)
    v0 = c.add_volume(nbytes=MB, tmp=MB)[1]
    v1 = c.add_volume(nbytes=MB, tmp=MB)[1]
    v2 = c.add_volume(nbytes=MB, tmp=MB)[1]
    _, a = c.submit(v0, [5] * 50, flags=DEVICE_POINTS | DEVICE_C)
    _, b = c.submit(v1, [5] * 50, flags=DEVICE_POINTS | DEVICE_C)
    for _ in range(2):
        c.step()   # both admitted, nothing completes
    c.lib.sim_complete(c.h, BUILD)
    c.step()
    _, d = c.submit(v2, [5] * 5, flags=DEVICE_POINTS | DEVICE_C)
    for _ in range(3):
        c.step()   # no completion of anything else: v2 cannot become resident
    assert c.state(d)[0] == PENDING and c.stats()["evictions"] == 0
    c.run()
    for r in (a, b, d):
        assert c.state(r)[:2] == (DONE, OK)


def test_no_eviction_when_it_cannot_make_room(core):
    # an idle resident volume is not evicted while the head request waits for an admitted one
    # while a (2.86 MB) is admitted: about 2 MB free + 256 KB evictable < 2.86 MB needed by b
    c = core(budget=5 * MB + 512 * KB, tick_points=100, chunk_points=50)
    v0 = c.add_volume(nbytes=256 * KB, tmp=256 * KB)[1]
    v1 = c.add_volume(nbytes=256 * KB, tmp=256 * KB)[1]
    _, r = c.submit(v1, [5] * 5, flags=DEVICE_POINTS | DEVICE_C)
    c.run()                                          # v1 resident and idle
    _, a = c.submit(v0, [1000] * 250)                # 3 MB of points, admitted
    _, b = c.submit(v0, [1000] * 250)                # waits for a: evicting v1 (256 KB) cannot help
    for _ in range(4):
        c.step()
    assert c.state(b)[0] == PENDING and c.stats()["evictions"] == 0
    c.run()
    assert c.state(b)[:2] == (DONE, OK) and c.stats()["evictions"] == 0


def test_cancel_pending_and_active(core):
    c = core(budget=4 * MB + 512 * KB, tick_points=100, chunk_points=50, ticks_in_flight=1)
    _, v = c.add_volume(nbytes=MB, tmp=MB)
    _, a = c.submit(v, [10] * 10000)   # 1.2 MB of points
    _, b = c.submit(v, [10] * 10)
    _, big = c.submit(v, [1000] * 200)   # 2.4 MB: waits behind a
    for _ in range(4):
        c.step(complete=-1)
    assert c.state(big)[0] == PENDING
    assert c.lib.sim_cancel(c.h, big) == OK
    assert c.state(big)[:2] == (DONE, ECANCELED)
    # cancel a while it is being counted: nothing new is issued for it afterwards
    assert c.state(a)[0] == ACTIVE
    ch_before = c.chunks()
    n_a_before = (ch_before[:, 1] == a).sum()
    assert c.lib.sim_cancel(c.h, a) == OK
    c.run()
    ch = c.chunks()
    assert (ch[:, 1] == a).sum() <= n_a_before + 0
    assert c.state(a)[:2] == (DONE, ECANCELED)
    assert c.state(b)[:2] == (DONE, OK)
    assert not any(o[0] == FINAL and o[1] == a for o in c.ops())
    s = c.stats()
    assert s["used"] == _rup(MB) and s["live_tokens"] == 0
    assert c.lib.sim_cancel(c.h, a) == EINVAL      # finished
    assert c.lib.sim_cancel(c.h, 99999) == EINVAL  # unknown


def test_active_cancel_waits_for_issued_work(core):
    c = core(tick_points=100, chunk_points=50, ticks_in_flight=2)
    _, v = c.add_volume()
    _, a = c.submit(v, [10] * 100)
    for _ in range(3):
        c.step()              # uploads and ticks issued, none completed
    c.lib.sim_complete(c.h, BUILD)
    c.lib.sim_complete(c.h, BEGIN)
    c.lib.sim_complete(c.h, UPLOAD)
    c.step()
    c.step()
    c.lib.sim_cancel(c.h, a)
    c.step()
    assert c.state(a)[0] == ACTIVE     # a launch that uses it is still in flight
    c.lib.sim_complete(c.h, -1)
    c.step()
    assert c.state(a)[:2] == (DONE, ECANCELED)


@pytest.mark.parametrize("kind", [BUILD, BEGIN, UPLOAD, TICK, FINAL])
@pytest.mark.parametrize("when", ["issue", "done"])
def test_failure_fails_every_request(core, kind, when):
    c = core(tick_points=100, chunk_points=50)
    _, v = c.add_volume()
    rids = [c.submit(v, [10] * 30)[1] for _ in range(3)]
    if when == "issue":
        c.lib.sim_fail_issue(c.h, kind, EHIP)
    else:
        c.lib.sim_fail_done(c.h, kind)
    for _ in range(200):
        c.step(complete=-1)
        if c.stats()["failed"]:
            break
    assert c.stats()["failed"] == EHIP
    for r in rids:
        assert c.state(r)[:2] == (DONE, EHIP)
    assert c.submit(v, [1, 2])[0] == EHIP
    assert c.add_volume()[0] == EHIP


def test_submit_checks(core):
    c = core()
    _, v = c.add_volume()
    assert c.submit(v + 5, [1, 2])[0] == EINVAL
    assert c.submit(v, offsets=[1, 2, 3])[0] == ERANGE
    assert c.submit(v, offsets=[0, 5, 3, 2, -1])[0] == ERANGE   # offsets[S] < 0
    assert c.submit(v, [1], flags=8)[0] == EINVAL
    # a decrease inside is found by the set-up's check: the request ends with ERANGE, never counted,
    # and its host points are uploaded only within [0, P)
    rc, bad = c.submit(v, offsets=[0, 5, 3, 9])
    assert rc == OK
    c.run()
    assert c.state(bad)[:2] == (DONE, ERANGE)
    assert not any(o[0] == FINAL and o[1] == bad for o in c.ops())
    ch = c.chunks()
    assert len(ch) == 0 or bad not in ch[:, 1]
    rc, rid = c.submit(v, offsets=[0])
    assert rc == OK
    c.run()
    assert c.state(rid)[:2] == (DONE, OK) and c.state(rid)[2] == 0   # S = 0: no launch, C still written
    assert any(o[0] == FINAL and o[1] == rid for o in c.ops())


def test_device_points_are_not_uploaded(core):
    c = core(tick_points=100, chunk_points=50)
    _, v = c.add_volume(N=10, M=4)
    _, rid = c.submit(v, [10] * 30, flags=DEVICE_POINTS)
    c.run()
    assert not any(o[0] == UPLOAD for o in c.ops())
    begin = [o for o in c.ops() if o[0] == BEGIN][0]
    assert begin[4] == -1 and begin[2] >= 0 and begin[3] >= 0   # no points block, C and offsets held
    _, r2 = c.submit(v, [10] * 30, flags=DEVICE_C)
    c.run()
    begin = [o for o in c.ops() if o[0] == BEGIN][1]
    assert begin[2] == -1 and begin[4] >= 0


def test_stop_cancels_everything(core):
    c = core(tick_points=100, chunk_points=50, max_active=1)
    _, v = c.add_volume()
    rids = [c.submit(v, [10] * 30)[1] for _ in range(4)]
    for _ in range(3):
        c.step()
    c.lib.sim_stop(c.h)
    assert c.submit(v, [1])[0] == EBUSY
    c.run()
    states = [c.state(r) for r in rids]
    assert all(s[0] == DONE for s in states)
    assert states[-1][1] == ECANCELED


# ---------------------------------------------------------------------------------------------
# threaded wrapper
def test_service_threads_wait_and_timeout(sim):
    h = sim.svc_create(64 * MB, 1000, 100, 8, 2)
    try:
        vid = i32()
        assert sim.svc_add_volume(h, 10, 4, MB, ctypes.byref(vid)) == OK
        keep = []
        ids = []
        lock = threading.Lock()

        def client(seed):
            rng = np.random.default_rng(seed)
            for _ in range(20):
                off = np.concatenate([[0], np.cumsum(rng.integers(0, 50, size=int(rng.integers(0, 80))))]).astype(np.int64)
                rid = u64()
                assert sim.svc_submit(h, vid.value, off.ctypes.data, len(off) - 1, ctypes.byref(rid)) == OK
                with lock:
                    keep.append(off)
                    ids.append(rid.value)

        ths = [threading.Thread(target=client, args=(s,)) for s in range(4)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        ts, td = i64(), i64()
        for rid in ids:
            assert sim.svc_wait(h, rid, 5_000_000, ctypes.byref(ts), ctypes.byref(td)) == OK
            assert td.value >= ts.value > 0
            assert sim.svc_wait(h, rid, 0, ctypes.byref(ts), ctypes.byref(td)) == EINVAL   # record dropped
    finally:
        sim.svc_destroy(h)


def test_service_timeout_cancel_and_shutdown(sim):
    h = sim.svc_create(64 * MB, 100, 50, 8, 200_000)   # every operation takes 200k polls
    try:
        vid = i32()
        sim.svc_add_volume(h, 10, 4, MB, ctypes.byref(vid))
        off = np.arange(0, 1001, 10, dtype=np.int64)
        rid = u64()
        assert sim.svc_submit(h, vid.value, off.ctypes.data, len(off) - 1, ctypes.byref(rid)) == OK
        ts, td = i64(), i64()
        assert sim.svc_wait(h, rid.value, 20_000, ctypes.byref(ts), ctypes.byref(td)) == ETIMEDOUT
        rid2 = u64()
        assert sim.svc_submit(h, vid.value, off.ctypes.data, len(off) - 1, ctypes.byref(rid2)) == OK
    finally:
        sim.svc_destroy(h)   # cancels both and drains (the simulated operations finish eventually)
