"""The batched and served forms at the sizes of their benchmark workloads, against the oracle.

* The 32-subject batched workload (grids between 64^3 and 145x174x145, N 5k-45k, M in {70,180,360},
  S 100k-2M per subject, 2.37G points in all): one plan with the default schedule and one tuned,
  every subject's C compared element by element with the oracle (Alg. 2, Section 2).  The oracle
  runs subject by subject on 2^16-streamline ranges in parallel threads and sums them: C is additive
  over streamline subsets, which the CPU suite pins.
* The served mix: 64^3 requests (S = 10k), 1.25 mm requests (S = 1M), and super-resolution requests
  (1.25 mm walks, S = 1M, scaled by fl32(1.25/0.7) onto the 0.7 mm volumes; one with a point
  inserted between neighbours, Section 3), plus a 1.25 mm request in the end-label mode, all in
  flight together with host points and host C, each compared with the oracle.
"""
import os
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth

pytestmark = pytest.mark.gpu


def _workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _oracle(w, scale=1.0, mode=0, upsample=1):
    pts = w.points.cpu().numpy() if isinstance(w.points, torch.Tensor) else w.points
    off = w.offsets.cpu().numpy()
    roi = w.roi.cpu().numpy() if isinstance(w.roi, torch.Tensor) else w.roi
    lab = w.lab.cpu().numpy() if isinstance(w.lab, torch.Tensor) else w.lab
    return oracle.count_chunked(pts, off, roi, lab, w.N, w.M, scale=scale, streamlines_per_chunk=1 << 16,
                                workers=_workers(), mode=mode, upsample=upsample)


def test_32_subject_plan_default_and_tuned(fc, tmp_path):
    t0 = time.time()
    subs, expect = [], []
    for k in range(32):
        w = synth.make_batch_subject(k, device="cuda")
        subs.append(dict(points=w.points, offsets=w.offsets, roi=w.roi, lab=w.lab, N=w.N, M=w.M, scale=1.0,
                         C=torch.full((w.N, w.M), -1, dtype=torch.int32, device="cuda")))
        expect.append(_oracle(w))          # one subject's points on the host at a time
        print(f"subject {k}: dims {w.dims} N={w.N} M={w.M} S={w.S} P={w.P} pairs={int(expect[-1].sum())} "
              f"({time.time() - t0:.0f}s)", flush=True)
    P = sum(int(d["points"].shape[0]) for d in subs)
    assert P > 2_000_000_000
    for tune in (False, True):
        plan = fc.Plan(subs, tune=tune, tune_cache=str(tmp_path / "tune.txt") if tune else None)
        for d in subs:
            d["C"].fill_(-1)
        plan.launch()
        torch.cuda.synchronize()
        print(f"plan tune={tune} schedule {plan.schedule}", flush=True)
        for k, (d, e) in enumerate(zip(subs, expect)):
            np.testing.assert_array_equal(d["C"].cpu().numpy(), e, err_msg=f"subject {k} tune={tune}")
        plan.close()


def test_served_mix_at_full_size(fc):
    t0 = time.time()
    vA, vB, vC = synth.volumes_tiny64(), synth.volumes_125mm(2), synth.volumes_07mm(3)
    srv = fc.Server(memory_budget=24 << 30)
    vid = {"64^3": srv.add_volume(vA.roi, vA.lab, vA.N, vA.M), "1.25mm": srv.add_volume(vB.roi, vB.lab, vB.N, vB.M),
           "sr": srv.add_volume(vC.roi, vC.lab, vC.N, vC.M)}
    vols = {"64^3": vA, "1.25mm": vB, "sr": vC}
    # (shape, seed, S, scale, mode, upsample)
    mix = [("64^3", 5000, 10_000, 1.0, 0, 1), ("1.25mm", 5100, 1_000_000, 1.0, 0, 1),
           ("sr", 5102, 1_000_000, synth.SR_SCALE, 0, 1), ("64^3", 5001, 10_000, 1.0, 0, 1),
           ("1.25mm", 5101, 1_000_000, 1.0, 1, 1), ("sr", 5103, 1_000_000, synth.SR_SCALE, 0, 2),
           ("64^3", 5002, 10_000, 1.0, 0, 1), ("64^3", 5003, 10_000, 1.0, 0, 1)]
    reqs = []
    for shape, seed, S, scale, mode, up in mix:
        if shape == "64^3":
            w = synth.make_tiny64(seed=seed, S=S, device="cuda")
        else:
            w = synth.make_subject_walks(vB, seed, S, 150.0, 20, 600, "cuda", shape)
        v = vols[shape]
        pts = torch.empty(w.points.shape, dtype=torch.float32, pin_memory=True)
        pts.copy_(w.points)
        off = w.offsets.cpu()
        del w
        out = torch.full((v.N, v.M), -1, dtype=torch.int32, pin_memory=True)
        exp = oracle.count_chunked(pts.numpy(), off.numpy(), v.roi, v.lab, v.N, v.M, scale=scale,
                                   streamlines_per_chunk=1 << 16, workers=_workers(), mode=mode, upsample=up)
        reqs.append(dict(name=f"{shape} seed={seed} mode={mode} u={up}", pts=pts, off=off, out=out, exp=exp,
                         vid=vid[shape], scale=scale, mode=mode, up=up, P=int(pts.shape[0])))
        print(f"{reqs[-1]['name']}: S={S} P={reqs[-1]['P']} pairs={int(exp.sum())} ({time.time() - t0:.0f}s)", flush=True)
    rids = [srv.submit(r["vid"], r["pts"], r["off"], r["out"], scale=r["scale"], mode=r["mode"], upsample=r["up"])
            for r in reqs]
    for rid, r in zip(rids, reqs):
        info = srv.wait(rid, timeout=120)
        assert info["status"] == fc.OK, r["name"]
        np.testing.assert_array_equal(r["out"].numpy(), r["exp"], err_msg=r["name"])
    st = srv.stats()
    print(f"server: {st}", flush=True)
    assert st["failed"] == 0 and st["launches"] >= 2
    srv.close()
