"""Benchmark: pass-through connectivity counting on one MI355X.

One step = one fastcod_count call over the whole 0.7 mm-like subject (260x311x260 grid,
N about 45.8k ROI rows, M = 180 labels, S = 5M streamlines, about 1.1G points): the compact
volume build, the zero fill of C, the partition, the counting kernel and the overflow fallback,
with every input already resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0        # MI355X HBM3E peak
KERNEL_NAME = "k_count_stream4"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "count_stream_07mm_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t pairs from the HIP runtime (timing events on the counting kernel's own stream)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        rc = self.hip.hipEventCreate(ctypes.byref(e))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed ({rc})")
        return e.value

    def elapsed_ms(self, a, b):
        self.hip.hipEventSynchronize(b)
        ms = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)

    def destroy(self, e):
        self.hip.hipEventDestroy(e)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "internal.h", "host.h", "api.hip"):
        with open(os.path.join(ROOT, "paper_2302_09247_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_per_launch():
    """HBM bytes per counting launch from committed rocprofv3 counters, if they match the source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_source_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_launch")


def host_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cpus_usable": len(os.sched_getaffinity(0)), "nproc": os.cpu_count()}


def oracle_workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_config_baselines(fastcod, synth, vols07, w07, C07):
    """The oracle on the 64^3 and 1.25 mm subjects (in full, 1 thread and all usable threads) and on the
    0.7 mm subject (in full on all usable threads), each result compared element by element with the
    GPU's C of the same input."""
    import numpy as np
    import torch
    import oracle
    workers = oracle_workers()
    rows = []
    for name, make in (("64^3", lambda: synth.make_tiny64(seed=1, S=10_000, device="cuda")),
                       ("1.25mm", lambda: synth.make_125mm(S=1_000_000, device="cuda"))):
        w = make()
        C = fastcod.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
        pts, off = w.points.cpu().numpy(), w.offsets.cpu().numpy()
        roi, lab = w.roi.cpu().numpy(), w.lab.cpu().numpy()
        t0 = time.perf_counter()
        e1 = oracle.count(pts, off, roi, lab, w.N, w.M)
        d1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        ea = oracle.count_chunked(pts, off, roi, lab, w.N, w.M, streamlines_per_chunk=1 << 14, workers=workers)
        da = time.perf_counter() - t0
        got = C.cpu().numpy().astype(np.int64)
        rows.append({"config": name, "S": w.S, "P": w.P, "points_per_s_1core": w.P / d1,
                     "points_per_s_all_cores": w.P / da, "threads": workers,
                     "bit_exact": bool(np.array_equal(got, e1) and np.array_equal(got, ea))})
        log(f"cpu oracle {name}: {w.P / d1:.3e} points/s (1 thread), {w.P / da:.3e} ({workers} threads), "
            f"bit_exact={rows[-1]['bit_exact']}")
        del w, C
    t0 = time.perf_counter()
    pts = w07.points.cpu().numpy()
    off = w07.offsets.cpu().numpy()
    t_copy = time.perf_counter() - t0
    t0 = time.perf_counter()
    e = oracle.count_chunked(pts, off, vols07.roi, vols07.lab, w07.N, w07.M, streamlines_per_chunk=1 << 16,
                             workers=workers)
    da = time.perf_counter() - t0
    ok = bool(np.array_equal(C07.cpu().numpy().astype(np.int64), e))
    rows.append({"config": "0.7mm", "S": w07.S, "P": w07.P, "points_per_s_1core": None,
                 "points_per_s_all_cores": w07.P / da, "threads": workers, "bit_exact": ok,
                 "note": f"1-thread rate: cpu_baseline (a 3M-streamline sample); points copied to the host in "
                         f"{t_copy:.1f} s (outside the timing)"})
    log(f"cpu oracle 0.7mm (whole subject): {w07.P / da:.3e} points/s on {workers} threads, bit_exact={ok}")
    return rows


def run_ceilings(fastcod, points, vol, scale=1.0, nwords_small=45808 * 180, reps=5) -> dict:
    """The ceiling probes (include/fastcod_probe.h) on this device: the read-only point stream and the
    stream plus every point's compact-volume lookups over `points`, and no-return int32 atomics at
    2^26 indices in three patterns -- uniform over a C of the 0.7 mm size (33 MB), uniform over 710 MB
    (the batched subjects' matrices together), and runs of 8 consecutive entries (one streamline's
    neighbouring ROI rows under one label in a transposed C) over 33 MB."""
    import torch
    ev = HipEvents()
    hip = ev.hip
    hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        a, b = ev.create(), ev.create()
        hip.hipEventRecord(a, stream.cuda_stream)
        for _ in range(reps):
            fn()
        hip.hipEventRecord(b, stream.cuda_stream)
        ms = ev.elapsed_ms(a, b) / reps
        ev.destroy(a)
        ev.destroy(b)
        return ms

    P = int(points.shape[0])
    out = {}
    ms = timed(lambda: fastcod.probe_stream(points))
    out["stream"] = {"ms": ms, "GBps": 12 * P / (ms * 1e-3) / 1e9, "bytes": 12 * P}
    ms = timed(lambda: fastcod.probe_lookup(vol, points, scale=scale))
    out["stream_lookup"] = {"ms": ms, "GBps": 12 * P / (ms * 1e-3) / 1e9, "points_per_s": P / (ms * 1e-3)}
    n = 1 << 26
    g = torch.Generator(device="cuda")
    g.manual_seed(123)
    pats = {}
    big = 710 * (1 << 20) // 4
    for name, nwords in (("random_33MB", nwords_small), ("random_710MB", big), ("runs8_33MB", nwords_small)):
        if name.startswith("runs8"):
            base = torch.randint(0, nwords // 8, (n // 8, 1), generator=g, device="cuda", dtype=torch.int64) * 8
            idx = (base + torch.arange(8, device="cuda")).reshape(-1).to(torch.int32)
        else:
            idx = torch.randint(0, nwords, (n,), generator=g, device="cuda", dtype=torch.int32)
        target = torch.zeros(nwords, dtype=torch.int32, device="cuda")
        ms = timed(lambda: fastcod.probe_atomics(target, idx))
        pats[name] = {"ms": ms, "atomics_per_s": n / (ms * 1e-3), "atomics": n, "target_bytes": 4 * nwords}
        del idx, target
    out["atomics"] = pats
    torch.cuda.empty_cache()
    for k, v in out.items():
        log(f"ceiling {k}: {v}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--streamlines", type=int, default=5_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form keys of the default line")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form keys of the default line")
    ap.add_argument("--cpu-sample-streamlines", type=int, default=3_000_000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for rocprofv3 counter scaling)")
    ap.add_argument("--form", choices=("plain", "batched", "served", "sr", "ceilings"), default="plain",
                    help="plain: the 0.7 mm subject (default); batched: many subjects in one graph launch; "
                         "served: Poisson request stream")
    ap.add_argument("--subjects", type=int, default=32)
    ap.add_argument("--served-subjects", type=int, default=8, help="resident subjects per request shape")
    ap.add_argument("--served-requests", type=int, default=200, help="requests per Poisson rate")
    ap.add_argument("--rates", default="0.1,0.25,0.5,0.75,0.9,1.0,1.2",
                    help="Poisson rates as fractions of the measured saturation throughput")
    ap.add_argument("--tune-cache", default=None)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the counting path runs on a single MI355X "
              "(a multi-GPU run would shard streamlines and all-reduce C; no multi-GPU path is implemented).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = 1 << 30   # 4 GiB read + 4 GiB written per copy
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {4 * n} bytes")
        return

    from paper_2302_09247_amd import fastcod, synth
    fastcod.load()
    if args.form == "batched":
        return bench_batched(args)
    if args.form == "served":
        return bench_served(args)
    if args.form == "sr":
        return bench_sr(args)
    if args.form == "ceilings":
        return bench_ceilings(args)
    t0 = time.time()
    vols = synth.volumes_07mm()
    log(f"volumes: N={vols.N} M={vols.M} dims={vols.dims} ({time.time() - t0:.1f}s)")
    t0 = time.time()
    w = synth.make_07mm(S=args.streamlines, device="cuda", vols=vols)
    torch.cuda.synchronize()
    S, P = w.S, w.P
    X, Y, Z = vols.dims
    log(f"workload: S={S} P={P} ({12 * P / 1e9:.2f} GB of points) generated in {time.time() - t0:.1f}s")

    ev = HipEvents()
    stream = torch.cuda.current_stream()
    C = torch.empty((w.N, w.M), dtype=torch.int32, device="cuda")
    for i in range(args.warmup):
        fastcod.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=stream)
    torch.cuda.synchronize()

    evs = [(ev.create(), ev.create()) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        fastcod.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, out=C, stream=stream, events=evs[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    kernel_ms = [ev.elapsed_ms(a, b) for a, b in evs]
    for a, b in evs:
        ev.destroy(a)
        ev.destroy(b)
    pair_total = int(C.sum(dtype=torch.int64).item())

    ms_per_step = 1e3 * elapsed / args.steps
    value = P * args.steps / elapsed
    k_ms = sum(kernel_ms) / len(kernel_ms)
    # algorithmic bytes of one step: points, offsets, both volumes read once, C written once
    alg_bytes = 12 * P + 8 * (S + 1) + 8 * X * Y * Z + 4 * w.N * w.M
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    log(f"step {ms_per_step:.3f} ms, {KERNEL_NAME} avg {k_ms:.3f} ms (min {min(kernel_ms):.3f}), "
        f"{achieved:.0f} GB/s algorithmic, pairs {pair_total}")

    # the same step against a resident compact volume (built once, outside the timed region): zero-fill,
    # partition, count, fallback and histogram only, the per-subject step when volumes are reused
    vol = fastcod.Volume(w.roi, w.lab, w.N, w.M, stream=stream)
    Cr = torch.empty_like(C)
    for _ in range(max(args.warmup, 1)):
        vol.count(w.points, w.offsets, out=Cr, stream=stream)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        vol.count(w.points, w.offsets, out=Cr, stream=stream)
    torch.cuda.synchronize()
    res_elapsed = time.perf_counter() - t_start
    if not torch.equal(Cr, C):
        raise SystemExit("resident-volume count differs from the plain count")
    res_ms = 1e3 * res_elapsed / args.steps
    resident = {"ms_per_step": res_ms, "value": P * args.steps / res_elapsed,
                "unit": "points/s", "step": "partition (zeroes C) + count + overflow fallback + pair histogram (volume resident)"}
    vol.close()
    del Cr
    log(f"resident-volume step {res_ms:.3f} ms")

    vol = fastcod.Volume(w.roi, w.lab, w.N, w.M, stream=stream)
    ceilings = run_ceilings(fastcod, w.points, vol)
    vol.close()

    # the parcellation outputs of this C (single-colour labels, pie-glyph fractions, row sums)
    pa = []
    for i in range(6):
        a, b = ev.create(), ev.create()
        fastcod.parcellate(C, stream=stream, events=(a, b))
        if i >= 2:
            pa.append(ev.elapsed_ms(a, b))
        ev.destroy(a)
        ev.destroy(b)
    p_ms = sum(pa) / len(pa)
    p_bytes = 8 * w.N * w.M + 12 * w.N
    parcellate = {"kernel": "k_parcellate", "ms": p_ms, "bytes": p_bytes, "GBps": p_bytes / (p_ms * 1e-3) / 1e9,
                  "frac_of_peak": p_bytes / (p_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
    log(f"parcellate: {p_ms * 1e3:.1f} us, {parcellate['GBps']:.0f} GB/s")

    # stream-copy ceiling on this device: a 4 GiB device-to-device copy (read + write bytes / time)
    ca = torch.empty(1 << 30, dtype=torch.float32, device="cuda")
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * 4 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb
    log(f"device copy: {copy_gbps:.0f} GB/s (read + write)")

    cpu = cpu_parallel = None
    cpu_configs = None
    bit_exact = None
    if not args.no_cpu_baseline:
        import numpy as np
        import oracle
        ns = min(args.cpu_sample_streamlines, S)
        p_end = int(w.offsets[ns].item())
        # the GPU's C of the same sample, for the element-by-element check
        Cs = fastcod.count(w.points[:p_end], w.offsets[:ns + 1].contiguous(), w.roi, w.lab, w.N, w.M)
        got = Cs.cpu().numpy().astype(np.int64)
        del Cs
        pts = w.points[:p_end].cpu().numpy()
        off = w.offsets[:ns + 1].cpu().numpy()
        roi, lab = vols.roi, vols.lab
        t0 = time.perf_counter()
        exp = oracle.count(pts, off, roi, lab, w.N, w.M)
        dt = time.perf_counter() - t0
        sample_exact = bool(np.array_equal(got, exp))
        cpu = {"value": p_end / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
               "sample": f"first {ns} of {S} streamlines ({p_end} points) of the same workload, "
                         f"single-threaded C oracle, {dt:.1f} s",
               "bit_exact": sample_exact, **host_info()}
        log(f"cpu oracle: {p_end / dt:.3e} points/s over {dt:.1f}s, GPU C of the sample bit-exact: {sample_exact}")
        # the same sample on all usable host cores (the oracle is additive over streamline ranges)
        workers = oracle_workers()
        t0 = time.perf_counter()
        exp2 = oracle.count_chunked(pts, off, roi, lab, w.N, w.M, streamlines_per_chunk=1 << 16, workers=workers)
        dtp = time.perf_counter() - t0
        cpu_parallel = {"value": p_end / dtp, "unit": "points/s", "cores": workers, "kind": "oracle",
                        "sample": f"the same {p_end} points, 2^16-streamline ranges on {workers} threads, {dtp:.1f} s",
                        "bit_exact": bool(np.array_equal(got, exp2))}
        log(f"cpu oracle on {workers} threads: {p_end / dtp:.3e} points/s over {dtp:.1f}s")
        del pts, off, exp, exp2, got
        cpu_configs = cpu_config_baselines(fastcod, synth, vols, w, C)
        bit_exact = sample_exact and all(r["bit_exact"] for r in cpu_configs)

    roofline = {"bound": "hbm", "kernel": KERNEL_NAME, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_per_launch(),
                "kernel_ms": k_ms, "algorithmic_bytes": alg_bytes,
                "bytes_model": "12 P + 8 (S+1) + 8 X Y Z + 4 N M",
                "frac_resident_step": alg_bytes / (res_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                "frac_step": alg_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                "pair_updates_per_s": pair_total / (k_ms * 1e-3),
                "copy_GBps": copy_gbps,
                "stream_ceiling_GBps": ceilings["stream"]["GBps"],
                "stream_lookup_ceiling_GBps": ceilings["stream_lookup"]["GBps"],
                "frac_of_stream_ceiling": (12 * P / (k_ms * 1e-3) / 1e9) / ceilings["stream"]["GBps"],
                "atomic_ceiling_per_s": ceilings["atomics"]["random_33MB"]["atomics_per_s"]}
    out = {
        "metric": "streamline points/s into bit-exact C[NxM]; HBM GB/s as % of MI355X peak",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "0.7mm-like subject: 260x311x260 grid, two-ellipsoid ROI, 180 shell labels, "
                               "random-walk streamlines (step 0.5 voxel, lognormal lengths median 270 in [30,1000])",
                   "S": S, "P": P, "N": w.N, "M": w.M, "pairs": pair_total,
                   "step": "compact volume build + partition (zeroes C) + count + overflow fallback + pair histogram",
                   "parallelism": "1 GPU"},
        "bit_exact": bit_exact,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_parallel,
        "cpu_baseline_configs": cpu_configs,
        "resident_volume": resident,
        "parcellate": parcellate,
        "ceilings": ceilings,
    }
    del w, C
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_batched:
        b = run_batched(args, fastcod, synth)
        out["batched"] = {k: b[k] for k in ("batched_ms", "plain_ms", "batched_over_plain", "bit_identical",
                                             "points_per_s", "plain_points_per_s", "algorithmic_GBps", "frac",
                                             "pair_updates_per_s", "schedule", "S", "P")}
        # every pair update of the batched kernel is a no-return atomic into its subject's C
        out["batched"]["atomics_per_s"] = b["pair_updates_per_s"]
        out["batched"]["atomic_ceiling_per_s"] = ceilings["atomics"]["random_710MB"]["atomics_per_s"]
        torch.cuda.empty_cache()
    if not args.no_served:
        r = run_served(args, fastcod, synth, [0.5, 0.9])
        out["served"] = {"saturation_requests_per_s": r["saturation"],
                         "points_per_s_at_saturation": r["points_per_s_at_saturation"],
                         "rates": [{k: row[k] for k in ("rate_frac", "rate", "p50_ms", "p99_ms", "throughput")}
                                   for row in r["sweep"]],
                         "bit_identical": r["bit_identical"], "requests_per_rate": args.served_requests}
    print(json.dumps(out), flush=True)


def run_batched(args, fastcod, synth) -> dict:
    """All subjects of the batched workload counted by one tuned, graph-captured plan launch, against
    the same subjects counted one by one with resident volumes (plain path) on the same GPU."""
    import torch
    t0 = time.time()
    subs = []
    for k in range(args.subjects):
        w = synth.make_batch_subject(k, device="cuda")
        subs.append(dict(points=w.points, offsets=w.offsets, roi=w.roi, lab=w.lab, N=w.N, M=w.M, scale=1.0,
                         C=torch.empty((w.N, w.M), dtype=torch.int32, device="cuda"), dims=w.dims))
        log(f"subject {k}: dims {w.dims} N={w.N} M={w.M} S={w.S} P={w.P}")
    torch.cuda.synchronize()
    P = sum(int(d["points"].shape[0]) for d in subs)
    S = sum(int(d["offsets"].shape[0]) - 1 for d in subs)
    log(f"batched workload: {len(subs)} subjects, S={S} P={P} ({12 * P / 1e9:.1f} GB) in {time.time() - t0:.0f}s")
    t0 = time.time()
    plan = fastcod.Plan(subs, tune=True, tune_cache=args.tune_cache)
    log(f"plan (with tuning) built in {time.time() - t0:.1f}s, schedule {plan.schedule}")
    ev = HipEvents()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    a, b = ev.create(), ev.create()
    hip = ev.hip
    hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    hip.hipEventRecord(a, stream.cuda_stream)
    for _ in range(args.steps):
        plan.launch(stream)
    hip.hipEventRecord(b, stream.cuda_stream)
    batched_ms = ev.elapsed_ms(a, b) / args.steps
    batched_C = [d["C"].clone() for d in subs]
    # plain: resident volume per subject, one fastcod_volume_count call each
    vols = [fastcod.Volume(d["roi"], d["lab"], d["N"], d["M"]) for d in subs]
    torch.cuda.synchronize()
    outs = [torch.empty_like(d["C"]) for d in subs]
    for v, d, o in zip(vols, subs, outs):
        for _ in range(max(1, args.warmup)):
            v.count(d["points"], d["offsets"], out=o)
    torch.cuda.synchronize()
    plain_ms = 0.0
    for v, d, o in zip(vols, subs, outs):
        hip.hipEventRecord(a, stream.cuda_stream)
        for _ in range(args.steps):
            v.count(d["points"], d["offsets"], out=o)
        hip.hipEventRecord(b, stream.cuda_stream)
        plain_ms += ev.elapsed_ms(a, b) / args.steps
    identical = all(torch.equal(c, o) for c, o in zip(batched_C, outs))
    pairs = sum(int(c.sum(dtype=torch.int64).item()) for c in batched_C)
    sched = plan.schedule
    for v in vols:
        v.close()
    plan.close()
    vox = sum(d["dims"][0] * d["dims"][1] * d["dims"][2] for d in subs)
    nm = sum(d["N"] * d["M"] for d in subs)
    alg_bytes = 12 * P + 8 * (S + len(subs)) + 8 * vox + 4 * nm
    log(f"batched {batched_ms:.3f} ms per launch, plain sum {plain_ms:.3f} ms, identical={identical}")
    del subs, batched_C, outs
    return {"batched_ms": batched_ms, "plain_ms": plain_ms, "batched_over_plain": plain_ms / batched_ms,
            "bit_identical": identical, "points_per_s": P / (batched_ms * 1e-3),
            "plain_points_per_s": P / (plain_ms * 1e-3), "algorithmic_bytes": alg_bytes,
            "algorithmic_GBps": alg_bytes / (batched_ms * 1e-3) / 1e9,
            "frac": alg_bytes / (batched_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "pair_updates_per_s": pairs / (batched_ms * 1e-3), "pairs": pairs, "schedule": sched, "S": S, "P": P,
            "subjects": args.subjects}


def bench_batched(args):
    from paper_2302_09247_amd import fastcod, synth
    r = run_batched(args, fastcod, synth)
    out = {
        "metric": "batched streamline points/s (all subjects, one graph launch) vs the plain per-subject path",
        "value": r["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["batched_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{r['subjects']} subjects, grids between 64^3 and 145x174x145, N 5k-45k, "
                               f"M in {{70,180,360}}, S 100k-2M", "S": r["S"], "P": r["P"], "pairs": r["pairs"],
                   "schedule": r["schedule"]},
        "algorithmic_GBps": r["algorithmic_GBps"], "frac": r["frac"], "pair_updates_per_s": r["pair_updates_per_s"],
        "plain_value": r["plain_points_per_s"], "plain_ms": r["plain_ms"],
        "batched_over_plain": r["batched_over_plain"], "bit_identical": r["bit_identical"],
    }
    print(json.dumps(out), flush=True)


def bench_ceilings(args):
    """The ceiling probes alone on the 0.7 mm subject's points and volumes (for rocprofv3)."""
    import torch
    from paper_2302_09247_amd import fastcod, synth
    w = synth.make_07mm(S=args.streamlines, device="cuda")
    vol = fastcod.Volume(w.roi, w.lab, w.N, w.M)
    torch.cuda.synchronize()
    c = run_ceilings(fastcod, w.points, vol)
    vol.close()
    out = {"metric": "ceiling probes: read-only point stream, stream + compact-volume lookups (GB/s of points), "
                     "no-return int32 atomics/s", "value": c["stream"]["GBps"], "unit": "GB/s", "n_gpus": 1,
           "steps": 5, "warmup": 1, "ms_per_step": c["stream"]["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "0.7mm-like subject points (S=5M) and volumes; 2^26 atomics per pattern",
                      "P": w.P}, "ceilings": c}
    print(json.dumps(out), flush=True)


def bench_sr(args):
    """Calls of one million streamlines: the 1.25 mm subject (u = 1), and the super-resolution job
    (Section 3): 1.25 mm streamlines (0.5-voxel steps) scaled by fl32(1.25/0.7) onto the 0.7 mm
    volumes, counted as given (u = 1) and with one point inserted between neighbours (u = 2,
    0.45-voxel spacing on the fine grid).  HBM bytes per point are the same 12 for every row: the
    inserted points never leave registers.  Bytes: 12 P + 8 (S+1) + 8 X Y Z + 4 N M."""
    import torch
    from paper_2302_09247_amd import fastcod, synth
    ev = HipEvents()
    stream = torch.cuda.current_stream()
    rows = []
    for name, make, ups in (("1.25mm", lambda: synth.make_125mm(S=1_000_000, device="cuda"), (1,)),
                            ("sr", lambda: synth.make_sr(S=1_000_000, device="cuda"), (1, 2))):
        w = make()
        torch.cuda.synchronize()
        X, Y, Z = w.dims
        C = torch.empty((w.N, w.M), dtype=torch.int32, device="cuda")
        for u in ups:
            for _ in range(args.warmup):
                fastcod.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=w.scale, upsample=u, out=C,
                              stream=stream)
            ks = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                a, b = ev.create(), ev.create()
                fastcod.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M, scale=w.scale, upsample=u, out=C,
                              stream=stream, events=(a, b))
                ks.append((a, b))
            torch.cuda.synchronize()
            step = (time.perf_counter() - t0) / args.steps
            kms = sum(ev.elapsed_ms(a, b) for a, b in ks) / len(ks)
            pairs = int(C.sum(dtype=torch.int64).item())
            alg = 12 * w.P + 8 * (w.S + 1) + 8 * X * Y * Z + 4 * w.N * w.M
            rows.append({"workload": name, "upsample": u, "S": w.S, "P": w.P, "ms_per_step": step * 1e3,
                         "kernel_ms": kms, "points_per_s": w.P / step,
                         "counted_points_per_s": (w.P + (u - 1) * (w.P - w.S)) / step, "pairs": pairs,
                         "algorithmic_bytes": alg, "kernel_GBps": alg / (kms * 1e-3) / 1e9,
                         "kernel_frac": alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBPS})
            log(f"{name} u={u}: step {step * 1e3:.3f} ms, kernel {kms:.3f} ms, {rows[-1]['kernel_GBps']:.0f} GB/s "
                f"({rows[-1]['kernel_frac']:.3f} of peak), pairs {pairs}")
        del w, C
        torch.cuda.empty_cache()
    out = {"metric": "streamline points/s of one-million-streamline calls (1.25 mm subject; SR job on the 0.7 mm grid)",
           "value": rows[0]["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": rows[0]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "1.25mm subject S=1M (145x174x145, N=8058, M=70); SR job: S=1M 1.25 mm walks x "
                                  "fl32(1.25/0.7) on 260x311x260, N=45.8k, M=180"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def run_served(args, fastcod, synth, rates) -> dict:
    """Served form: a request server with resident volumes receives a Poisson stream of requests --
    37.5% 64^3-grid subjects (10k streamlines), 37.5% 1.25 mm-grid subjects (1M streamlines), 25%
    super-resolution jobs (1.25 mm streamlines scaled by fl32(1.25/0.7) onto the 0.7 mm volumes).
    Streamlines of `served_subjects` subjects per shape are resident on the device; C goes to pinned
    host memory.  Latency = time C is in host memory minus the scheduled arrival.  Every result is
    compared with the same subject counted alone by the plain path."""
    import threading
    import numpy as np
    import torch
    t0 = time.time()
    ns = args.served_subjects
    vA, vB, vC = synth.volumes_tiny64(), synth.volumes_125mm(2), synth.volumes_07mm(3)
    subs = {"64^3": [synth.make_tiny64(seed=5000 + k, S=10_000, device="cuda") for k in range(ns)],
            "1.25mm": [synth.make_125mm(seed=5100 + k, S=1_000_000, device="cuda", vols=vB) for k in range(ns)]}
    torch.cuda.synchronize()
    log(f"served workload generated in {time.time() - t0:.0f}s")
    vols = {"64^3": (vA, 1.0), "1.25mm": (vB, 1.0), "sr": (vC, synth.SR_SCALE)}
    srv = fastcod.Server(memory_budget=48 << 30)
    vid = {k: srv.add_volume(v.roi, v.lab, v.N, v.M) for k, (v, _) in vols.items()}
    # solo results (plain path) and pinned host offsets
    solo, offs = {}, {}
    dev_vol = {k: (torch.from_numpy(v.roi).cuda(), torch.from_numpy(v.lab).cuda()) for k, (v, _) in vols.items()}
    for kind in ("64^3", "1.25mm", "sr"):
        src = "1.25mm" if kind == "sr" else kind
        v, scale = vols[kind]
        for k in range(ns):
            w = subs[src][k]
            C = fastcod.count(w.points, w.offsets, dev_vol[kind][0], dev_vol[kind][1], v.N, v.M, scale=scale)
            solo[(kind, k)] = C.cpu().numpy()
            if (src, k) not in offs:
                o = torch.empty(w.offsets.shape, dtype=torch.int64, pin_memory=True)
                o.copy_(w.offsets)
                offs[(src, k)] = o
    del dev_vol
    pts_per = {kind: float(np.mean([subs["1.25mm" if kind == "sr" else kind][k].P for k in range(ns)]))
               for kind in vols}
    pools = {kind: [] for kind in vols}

    def run(rate, nreq, seed):
        """nreq requests at Poisson `rate` (requests/s; None = all at once).  Returns per-request records."""
        rng = np.random.default_rng(seed)
        kinds = rng.choice(["64^3", "1.25mm", "sr"], size=nreq, p=[0.375, 0.375, 0.25])
        subj = rng.integers(0, ns, size=nreq)
        gaps = rng.exponential(1.0 / rate, size=nreq) if rate else np.zeros(nreq)
        arrive = np.cumsum(gaps) - gaps[0]
        need = {kind: int((kinds == kind).sum()) for kind in vols}
        for kind, n in need.items():   # pinned result buffers, one per request of the run
            v = vols[kind][0]
            while len(pools[kind]) < n:
                pools[kind].append(torch.empty((v.N, v.M), dtype=torch.int32, pin_memory=True))
        used = {kind: 0 for kind in vols}
        outs = []
        for i in range(nreq):
            outs.append(pools[kinds[i]][used[kinds[i]]])
            used[kinds[i]] += 1
        recs = [None] * nreq
        rids = [None] * nreq
        ready = threading.Semaphore(0)

        def collect():
            for i in range(nreq):
                ready.acquire()
                info = srv.wait(rids[i])
                recs[i] = (info, bool(np.array_equal(outs[i].numpy(), solo[(kinds[i], int(subj[i]))])))

        for i in range(nreq):
            outs[i].fill_(-1)          # a request that wrote nothing cannot match an earlier result
        th = threading.Thread(target=collect)
        th.start()
        start = time.monotonic_ns() + 2_000_000
        for i in range(nreq):
            due = start + int(arrive[i] * 1e9)
            while True:
                now = time.monotonic_ns()
                if now >= due:
                    break
                time.sleep(min(0.001, (due - now) / 1e9))
            src = "1.25mm" if kinds[i] == "sr" else kinds[i]
            w = subs[src][subj[i]]
            rids[i] = srv.submit(vid[kinds[i]], w.points, offs[(src, int(subj[i]))], outs[i], scale=vols[kinds[i]][1])
            ready.release()
        th.join()
        lat = np.array([(r[0]["t_done_ns"] - (start + int(a * 1e9))) / 1e6 for r, a in zip(recs, arrive)])
        span = (max(r[0]["t_done_ns"] for r in recs) - start) / 1e9
        ok = all(r[0]["status"] == 0 for r in recs)
        exact = all(r[1] for r in recs)
        pts = sum(pts_per[k] for k in kinds)
        return {"lat": lat, "span_s": span, "ok": ok, "exact": exact, "points": pts}

    run(None, 24, 99)   # warm-up: builds every volume
    burst = run(None, args.served_requests, 1)
    sat = args.served_requests / burst["span_s"]
    log(f"saturation: {sat:.1f} requests/s ({burst['points'] / burst['span_s']:.3e} points/s), "
        f"exact={burst['exact']} ok={burst['ok']}")
    sweep = []
    exact = burst["exact"] and burst["ok"]
    for j, frac in enumerate(rates):
        r = run(frac * sat, args.served_requests, 10 + j)
        exact &= r["exact"] and r["ok"]
        row = {"rate_frac": frac, "rate": frac * sat, "p50_ms": float(np.percentile(r["lat"], 50)),
               "p99_ms": float(np.percentile(r["lat"], 99)),
               "throughput": args.served_requests / r["span_s"], "exact": r["exact"] and r["ok"]}
        sweep.append(row)
        log(f"rate {frac:.2f}x = {row['rate']:.1f}/s: p50 {row['p50_ms']:.2f} ms p99 {row['p99_ms']:.2f} ms, "
            f"{row['throughput']:.1f} req/s, exact={row['exact']}")
    st = srv.stats()
    srv.close()
    return {"saturation": sat, "points_per_s_at_saturation": burst["points"] / burst["span_s"], "sweep": sweep,
            "bit_identical": exact, "server": st, "subjects": ns}


def bench_served(args):
    from paper_2302_09247_amd import fastcod, synth
    r = run_served(args, fastcod, synth, [float(x) for x in args.rates.split(",")])
    sat = r["saturation"]
    out = {
        "metric": "served requests/s at saturation (Poisson request stream, resident volumes, C to pinned host); "
                  "p50/p99 latency per rate",
        "value": sat, "unit": "requests/s", "n_gpus": 1, "steps": args.served_requests, "warmup": 24,
        "ms_per_step": 1e3 / sat, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"37.5% 64^3 (S=10k), 37.5% 1.25 mm (S=1M), 25% SR 1.25->0.7 mm; "
                               f"{r['subjects']} resident subjects per shape", "requests_per_rate": args.served_requests},
        "points_per_s_at_saturation": r["points_per_s_at_saturation"],
        "sweep": r["sweep"], "bit_identical": r["bit_identical"], "server": r["server"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
