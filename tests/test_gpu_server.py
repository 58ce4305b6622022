"""GPU tests of the served form (fastcod_server_*): every request's C must equal the oracle and the
plain single-call result, whatever else is in flight -- host or device points, host or device C,
several client threads, a budget small enough to force queueing and volume eviction, and
cancellations in the mix."""
import threading

import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth

pytestmark = pytest.mark.gpu

SR_SCALE = 1.7857143


def _overflow_workload():
    rng = np.random.default_rng(11)
    X, Y, Z = 200, 30, 20
    roi = np.arange(X * Y * Z, dtype=np.int32).reshape(Z, Y, X)
    lab = rng.integers(-1, 12, size=(Z, Y, X)).astype(np.int32)
    parts, off = [], [0]
    for _ in range(40):
        T = int(rng.integers(1, 900))
        o = np.array([rng.uniform(0, 20), rng.uniform(0, Y), rng.uniform(0, Z)])
        d = np.array([1.0, rng.normal() * 0.1, rng.normal() * 0.1])
        d /= np.linalg.norm(d)
        parts.append((o + np.arange(T)[:, None] * 0.5 * d).astype(np.float32))
        off.append(off[-1] + T)
    return synth.Workload("overflow", torch.from_numpy(np.concatenate(parts)), torch.from_numpy(np.array(off)),
                          torch.from_numpy(roi), torch.from_numpy(lab), X * Y * Z, 12)


@pytest.fixture(scope="module")
def cases():
    """(name, workload on the CPU, scale, expected C) -- expected from the oracle."""
    out = []
    w = synth.make_tiny64(seed=5, S=3000)
    out.append(("tiny64", w, 1.0))
    w = synth.make_batch_subject(3, S=4000)
    out.append(("subject3", w, 1.0))
    sm = synth.random_small(7, dims=(40, 30, 25), S=300, max_len=300)
    out.append(("scaled", sm, SR_SCALE))
    e = synth.make_tiny64(seed=6, S=10)
    out.append(("empty", synth.Workload("empty", torch.zeros((0, 3), dtype=torch.float32),
                                        torch.zeros(1, dtype=torch.int64), e.roi, e.lab, e.N, e.M), 1.0))
    out.append(("overflow", _overflow_workload(), 1.0))
    res = []
    for name, w, s in out:
        exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=s)
        res.append(dict(name=name, w=w, scale=s, expect=exp))
    return res


def _pinned(t):
    p = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    p.copy_(t)
    return p


def _submit(srv, vid, case, device_points, device_c):
    w = case["w"]
    pts = w.points.cuda() if device_points else _pinned(w.points)
    if device_c:
        out = torch.full((w.N, w.M), -5, dtype=torch.int32, device="cuda")
    else:
        out = torch.full((w.N, w.M), -5, dtype=torch.int32, pin_memory=True)
    rid = srv.submit(vid, pts, w.offsets, out, scale=case["scale"])
    return rid, out


def _register(srv, cases):
    return [srv.add_volume(c["w"].roi, c["w"].lab, c["w"].N, c["w"].M) for c in cases]


def test_requests_match_oracle_and_plain(fc, cases):
    srv = fc.Server(memory_budget=1 << 30, tick_points=1 << 16, chunk_points=1 << 12)
    vids = _register(srv, cases)
    pend = []
    for dp in (False, True):
        for dc in (False, True):
            for c, v in zip(cases, vids):
                rid, out = _submit(srv, v, c, dp, dc)
                pend.append((rid, out, c, dp, dc))
    for rid, out, c, dp, dc in pend:
        info = srv.wait(rid, timeout=60)
        assert info["status"] == fc.OK, (c["name"], dp, dc)
        np.testing.assert_array_equal(out.cpu().numpy(), c["expect"], err_msg=f"{c['name']} dp={dp} dc={dc}")
        assert info["t_done_ns"] >= info["t_admit_ns"] >= info["t_submit_ns"] > 0
    st = srv.stats()
    assert st["failed"] == 0 and st["active"] == 0 and st["pending"] == 0
    assert st["launches"] > len(cases)    # requests were cut into several launches
    srv.close()
    for c in cases:   # the plain single-call path gives the same C
        w = c["w"].to("cuda")
        plain = fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=c["scale"])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(plain.cpu().numpy(), c["expect"], err_msg=c["name"])


def test_concurrent_clients(fc, cases):
    srv = fc.Server(memory_budget=1 << 30, tick_points=1 << 15, chunk_points=1 << 11, max_active=6)
    vids = _register(srv, cases)
    errors = []

    def client(seed):
        rng = np.random.default_rng(seed)
        mine = []
        for _ in range(8):
            k = int(rng.integers(len(cases)))
            rid, out = _submit(srv, vids[k], cases[k], bool(rng.integers(2)), bool(rng.integers(2)))
            mine.append((rid, out, k))
        for rid, out, k in mine:
            info = srv.wait(rid, timeout=60)
            if info["status"] != fc.OK or not np.array_equal(out.cpu().numpy(), cases[k]["expect"]):
                errors.append((seed, cases[k]["name"], info["status"]))

    ths = [threading.Thread(target=client, args=(s,)) for s in range(3)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    assert not errors
    srv.close()


def test_small_budget_queues_and_evicts(fc, cases):
    c = cases[1]   # the largest grid
    w = c["w"]
    pts_d, out_d = w.points.cuda(), torch.empty((w.N, w.M), dtype=torch.int32, device="cuda")
    # resident bytes of its compact volume, as the server sizes it
    probe = fc.Server(memory_budget=1 << 30)
    v = probe.add_volume(w.roi, w.lab, w.N, w.M)
    assert probe.wait(probe.submit(v, pts_d, w.offsets, out_d), timeout=60)["status"] == fc.OK
    vol_bytes = probe.stats()["used_bytes"]
    probe.close()
    rup = lambda b: (b + 255) // 256 * 256
    nvox = w.roi.numel()
    build = vol_bytes + 2 * rup(4 * nvox) + rup(8 * (w.S + 1))
    # room for one build, but not for a build next to another resident copy of the volume
    srv = fc.Server(memory_budget=build + vol_bytes // 2, tick_points=1 << 15)
    va = srv.add_volume(w.roi, w.lab, w.N, w.M)
    vb = srv.add_volume(w.roi, w.lab, w.N, w.M)
    outs = []
    for vid in (va, vb, va, vb):
        o = torch.full((w.N, w.M), -1, dtype=torch.int32, device="cuda")
        outs.append((srv.submit(vid, pts_d, w.offsets, o), o))
    for rid, o in outs:
        assert srv.wait(rid, timeout=60)["status"] == fc.OK
        np.testing.assert_array_equal(o.cpu().numpy(), c["expect"])
    st = srv.stats()
    assert st["volume_builds"] == 4 and st["evictions"] == 3
    srv.close()


def test_budget_queueing_with_host_inputs(fc, cases):
    # host points and host C: about two of the largest requests fit at once, the rest queue
    w = cases[1]["w"]
    one = 12 * w.P + 4 * w.N * w.M
    srv = fc.Server(memory_budget=int(2.5 * one) + (64 << 20), tick_points=1 << 15, chunk_points=1 << 12)
    vids = _register(srv, cases)
    order = [1, 0, 1, 2, 1, 4, 1, 3, 0]
    pend = [(_submit(srv, vids[k], cases[k], False, False), k) for k in order]
    for (rid, out), k in pend:
        info = srv.wait(rid, timeout=60)
        assert info["status"] == fc.OK, cases[k]["name"]
        np.testing.assert_array_equal(out.numpy(), cases[k]["expect"], err_msg=cases[k]["name"])
    srv.close()


def test_cancel_in_the_mix(fc, cases):
    srv = fc.Server(memory_budget=1 << 30, tick_points=1 << 12, chunk_points=1 << 10)
    vids = _register(srv, cases)
    keep = []
    for k in (1, 0, 1, 2, 1):
        keep.append((_submit(srv, vids[k], cases[k], False, False), k))
    srv.cancel(keep[0][0][0])
    srv.cancel(keep[2][0][0])
    for i, ((rid, out), k) in enumerate(keep):
        info = srv.wait(rid, timeout=60)
        if i in (0, 2):
            assert info["status"] in (fc.OK, fc.ECANCELED)
            if info["status"] == fc.OK:
                np.testing.assert_array_equal(out.numpy(), cases[k]["expect"])
        else:
            assert info["status"] == fc.OK
            np.testing.assert_array_equal(out.numpy(), cases[k]["expect"], err_msg=cases[k]["name"])
    srv.close()


def test_submission_errors(fc, cases):
    srv = fc.Server(memory_budget=8 << 20)
    c = cases[0]
    v = srv.add_volume(c["w"].roi, c["w"].lab, c["w"].N, c["w"].M)
    out = torch.zeros((c["w"].N, c["w"].M), dtype=torch.int32)
    bad = c["w"].offsets.clone()
    bad[1] = 3
    with pytest.raises(fc.FastcodError) as e:   # offsets[0] != 0: refused at submission
        srv.submit(v, c["w"].points, bad + 1, out)
    assert e.value.status == fc.ERANGE
    # a decrease inside is found by the device check of the set-up: the request ends with ERANGE,
    # C_out untouched, and the server goes on serving
    bad = c["w"].offsets.clone()
    bad[2] = bad[1] - 1
    out.fill_(-7)
    rid = srv.submit(v, _pinned(c["w"].points), bad, out, scale=c["scale"])
    assert srv.wait(rid)["status"] == fc.ERANGE
    assert bool((out == -7).all())
    good = torch.zeros_like(out)
    assert srv.wait(srv.submit(v, _pinned(c["w"].points), c["w"].offsets, good, scale=c["scale"]))["status"] == 0
    np.testing.assert_array_equal(good.numpy().astype(np.int64), c["expect"])
    with pytest.raises(fc.FastcodError) as e:
        srv.submit(v + 7, c["w"].points, c["w"].offsets, out)
    assert e.value.status == fc.EINVAL
    big = torch.zeros((1 << 20, 3), dtype=torch.float32)
    with pytest.raises(fc.FastcodError) as e:   # 12 MB of host points can never fit 8 MB
        srv.submit(v, big, torch.tensor([0, 1 << 20]), out)
    assert e.value.status == fc.ENOMEM
    # the server still works
    rid = srv.submit(v, _pinned(c["w"].points), c["w"].offsets, out)
    assert srv.wait(rid, timeout=60)["status"] == fc.OK
    np.testing.assert_array_equal(out.numpy(), c["expect"])
    with pytest.raises(fc.FastcodError):
        srv.wait(rid)            # waited for already
    srv.close()


def test_requests_with_modes_and_upsampling(fc, cases):
    """Requests in the endpoint modes, Alg. 1's count and with point insertion, mixed in one server
    with pass-through ones, each against the oracle with its own options."""
    srv = fc.Server(memory_budget=1 << 30, tick_points=1 << 15, chunk_points=1 << 11)
    vids = _register(srv, cases)
    pend = []
    opts = [(1, 1), (2, 1), (3, 1), (0, 2), (0, 3), (0, 4), (0, 1)]
    for j, (mode, up) in enumerate(opts):
        for c, v in zip(cases, vids):
            w = c["w"]
            exp = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=c["scale"], mode=mode, upsample=up)
            dp = (j % 2) == 1
            pts = w.points.cuda() if dp else _pinned(w.points)
            out = torch.full((w.N, w.M), -5, dtype=torch.int32, pin_memory=True)
            rid = srv.submit(v, pts, w.offsets, out, scale=c["scale"], mode=mode, upsample=up)
            pend.append((rid, out, exp, f"{c['name']} mode={mode} u={up}"))
    for rid, out, exp, name in pend:
        info = srv.wait(rid, timeout=60)
        assert info["status"] == fc.OK, name
        np.testing.assert_array_equal(out.numpy(), exp, err_msg=name)
    assert sum(int(e.sum()) for _, _, e, _ in pend) > 0
    srv.close()


def test_request_options_are_checked(fc, cases):
    srv = fc.Server(memory_budget=64 << 20)
    c = cases[0]
    v = srv.add_volume(c["w"].roi, c["w"].lab, c["w"].N, c["w"].M)
    out = torch.zeros((c["w"].N, c["w"].M), dtype=torch.int32)
    for mode, up in ((4, 1), (1, 2), (0, 5)):
        with pytest.raises(fc.FastcodError) as e:
            srv.submit(v, _pinned(c["w"].points), c["w"].offsets, out, mode=mode, upsample=up)
        assert e.value.status == fc.EINVAL
    srv.close()


def test_device_inputs_ordered_after_the_callers_stream(fc, cases):
    """Device points and C written by work still in flight on the caller's stream at submission: the
    server's zero fill, counting and result must come after that work (regression: its streams used
    to ignore the caller's)."""
    c = cases[1]
    w = c["w"]
    srv = fc.Server(memory_budget=1 << 30, tick_points=1 << 15)
    v = srv.add_volume(w.roi, w.lab, w.N, w.M)
    src = w.points.cuda()
    busy = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    for rep in range(3):
        pts = torch.empty_like(src)
        out = torch.empty((w.N, w.M), dtype=torch.int32, device="cuda")
        with torch.cuda.stream(side):
            for _ in range(40):              # a long queue of work ahead of the writes
                busy.mul_(1.0000001)
            pts.copy_(src)
            out.fill_(-5)
            rid = srv.submit(v, pts, w.offsets, out)     # ordered after `side` (the current stream)
        info = srv.wait(rid, timeout=60)
        assert info["status"] == fc.OK
        np.testing.assert_array_equal(out.cpu().numpy(), c["expect"], err_msg=f"rep {rep}")
    srv.close()
