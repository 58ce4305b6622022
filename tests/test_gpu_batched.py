"""GPU tests of the batched form: one persistent, graph-captured launch over many subjects.

Each subject's C must be bit-identical to the plain single-subject call and to the oracle; the
captured graph is replayed several times with eager work in between, and every replay is checked.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth

pytestmark = pytest.mark.gpu


def _subject(w, device="cuda"):
    w = w.to(device)
    return dict(points=w.points, offsets=w.offsets, roi=w.roi, lab=w.lab, N=w.N, M=w.M, scale=w.scale,
                C=torch.full((w.N, w.M), -7, dtype=torch.int32, device=device), w=w)


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
def subjects():
    subs = []
    for k, S in ((0, 3000), (1, 9000), (2, 20000)):
        subs.append(_subject(synth.make_batch_subject(k, S=S, device="cuda")))
    subs.append(_subject(synth.make_tiny64(seed=3, S=2500, device="cuda")))
    sm = synth.random_small(5, dims=(30, 20, 25), S=200, max_len=200)
    subs.append(_subject(synth.Workload("scaled", sm.points, sm.offsets, sm.roi, sm.lab, sm.N, sm.M, 1.7857143)))
    empty = synth.make_tiny64(seed=4, S=10)
    subs.append(_subject(synth.Workload("empty", torch.zeros((0, 3), dtype=torch.float32),
                                        torch.zeros(1, dtype=torch.int64), empty.roi, empty.lab, empty.N, empty.M)))
    # shares the volume tensors of subject 0 (one compact volume for both)
    w0 = subs[0]["w"]
    other = synth.make_batch_subject(0, seed=9, S=4000, device="cuda", vols=synth.volumes_batch_subject(0))
    subs.append(dict(points=other.points, offsets=other.offsets, roi=w0.roi, lab=w0.lab, N=w0.N, M=w0.M, scale=1.0,
                     C=torch.zeros((w0.N, w0.M), dtype=torch.int32, device="cuda"),
                     w=synth.Workload("shared", other.points, other.offsets, w0.roi, w0.lab, w0.N, w0.M)))
    subs.append(_subject(_overflow_workload()))
    for d in subs:
        w = d["w"]
        d["expect"] = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=w.scale)
    return subs


def _check_all(subs):
    for d in subs:
        np.testing.assert_array_equal(d["C"].cpu().numpy(), d["expect"], err_msg=d["w"].name)


def test_plan_matches_oracle_and_plain(fc, subjects):
    plan = fc.Plan(subjects)
    plan.launch()
    torch.cuda.synchronize()
    _check_all(subjects)
    for d in subjects:
        plain = fc.count(d["points"], d["offsets"], d["roi"], d["lab"], d["N"], d["M"], scale=d["scale"])
        torch.cuda.synchronize()
        assert torch.equal(plain, d["C"]), d["w"].name
    plan.close()


def test_graph_replays_with_eager_work_between(fc, subjects):
    plan = fc.Plan(subjects)
    side = torch.cuda.Stream()
    for rep in range(3):
        for d in subjects:
            d["C"].fill_(12345)
        plan.launch()
        torch.cuda.synchronize()
        _check_all(subjects)
        # eager work of the program between replays: a plain count on another stream and torch ops
        with torch.cuda.stream(side):
            d = subjects[rep]
            fc.count(d["points"], d["offsets"], d["roi"], d["lab"], d["N"], d["M"], scale=d["scale"], stream=side)
            torch.cumsum(d["points"][:, 0], 0)
        torch.cuda.synchronize()
    # points are re-read by every launch: reversing every streamline leaves C unchanged, replacing the
    # points of one subject changes its C
    d = subjects[2]
    saved = d["points"].clone()
    d["points"].copy_(torch.flip(saved, dims=[0]))
    rev_off = (d["offsets"][-1] - torch.flip(d["offsets"], dims=[0])).contiguous()
    saved_off = d["offsets"].clone()
    d["offsets"].copy_(rev_off)
    plan.launch()
    torch.cuda.synchronize()
    _check_all(subjects)
    d["points"].copy_(saved)
    d["offsets"].copy_(saved_off)
    plan.close()


def test_tuner_and_cache(fc, subjects, tmp_path):
    cache = str(tmp_path / "tune.txt")
    plan = fc.Plan(subjects, tune=True, tune_cache=cache)
    sched = plan.schedule
    assert sched["tuned_ms"] > 0 and sched["batch"] in (2, 4)
    plan.launch()
    torch.cuda.synchronize()
    _check_all(subjects)
    plan.close()
    text = open(cache).read().split()
    assert len(text) == 5
    plan2 = fc.Plan(subjects, tune=True, tune_cache=cache)   # found in the cache: no new timing
    assert plan2.schedule["batch"] == sched["batch"] and plan2.schedule["items_per_wave"] == sched["items_per_wave"]
    assert len(open(cache).read().split()) == 5
    plan2.launch()
    torch.cuda.synchronize()
    _check_all(subjects)
    plan2.close()


def test_count_batched_one_shot(fc, subjects):
    for d in subjects:
        d["C"].fill_(-1)
    fc.count_batched(subjects)
    _check_all(subjects)


def test_subjects_sharing_one_C_receive_the_sum(fc):
    # two subjects on the same volumes writing one C_out (counted straight into it, no transposed
    # copy) and a third with a C of its own (counted through the transposed copy), in one plan,
    # launched twice: the shared C holds the sum of both subjects' counts after every launch
    a = synth.make_tiny64(seed=21, S=3000, device="cuda")
    b = synth.make_tiny64(seed=22, S=2000, device="cuda")
    c = synth.make_tiny64(seed=23, S=2500, device="cuda")
    shared = torch.full((a.N, a.M), -3, dtype=torch.int32, device="cuda")
    subs = [_subject(a), _subject(b), _subject(c)]
    subs[0]["C"] = shared
    subs[1]["C"] = shared
    exp_ab = sum(oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M) for w in (a, b))
    exp_c = oracle.count(c.points, c.offsets, c.roi, c.lab, c.N, c.M)
    assert exp_ab.sum() > 0 and exp_c.sum() > 0
    plan = fc.Plan(subs)
    for _ in range(2):
        plan.launch()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(shared.cpu().numpy(), exp_ab)
        np.testing.assert_array_equal(subs[2]["C"].cpu().numpy(), exp_c)


def test_plan_with_per_subject_options(fc):
    """Every kind of subject in one plan, each against the oracle with its own options: pass-through,
    the end label (Alg. 2 as printed), both end labels, Alg. 1's seed-to-end count, and point
    insertion with u = 2, 3, 4 (Section 3); the endpoint modes and upsampling also on the overflow
    workload, whose streamlines go through the batched fallback."""
    vols = [synth.volumes_batch_subject(k) for k in range(3)]
    specs = [(0, 1), (1, 1), (2, 1), (3, 1), (0, 2), (0, 3), (0, 4), (1, 1), (3, 1), (0, 1)]
    subs = []
    for j, (mode, up) in enumerate(specs):
        k = j % 3
        w = synth.make_batch_subject(k, seed=60 + j, S=2500 + 700 * j, device="cuda", vols=vols[k])
        d = _subject(w)
        d.update(mode=mode, upsample=up)
        subs.append(d)
    sr = synth.make_sr(seed=71, S=3000, device="cuda")
    for mode, up in ((0, 2), (2, 1)):
        d = _subject(sr)
        d.update(mode=mode, upsample=up)
        subs.append(d)
    for mode, up in ((1, 1), (2, 1), (0, 4)):
        d = _subject(_overflow_workload())
        d.update(mode=mode, upsample=up)
        subs.append(d)
    for d in subs:
        w = d["w"]
        d["expect"] = oracle.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=w.scale, mode=d["mode"],
                                   upsample=d["upsample"])
        assert d["expect"].sum() > 0, (w.name, d["mode"], d["upsample"])
    plan = fc.Plan(subs)
    for rep in range(2):
        for d in subs:
            d["C"].fill_(-3)
        plan.launch()
        torch.cuda.synchronize()
        for d in subs:
            np.testing.assert_array_equal(d["C"].cpu().numpy(), d["expect"],
                                          err_msg=f"{d['w'].name} mode={d['mode']} u={d['upsample']} rep={rep}")
    plan.close()
    for d in subs:   # the plain call with the same options agrees
        plain = fc.count(d["points"], d["offsets"], d["roi"], d["lab"], d["N"], d["M"], scale=d["scale"],
                         mode=d["mode"], upsample=d["upsample"])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(plain.cpu().numpy(), d["expect"])


def test_plan_rejects_bad_subject_options(fc):
    w = synth.make_tiny64(seed=8, S=100, device="cuda")
    for mode, up in ((4, 1), (1, 2), (0, 5), (-1, 1)):
        d = _subject(w)
        d.update(mode=mode, upsample=up)
        with pytest.raises(fc.FastcodError) as e:
            fc.Plan([d])
        assert e.value.status == fc.EINVAL
