"""Thin ctypes binding of libfastcod.so (C-ABI in include/fastcod.h).

Argument marshalling only: every step of the counting runs in the library's HIP kernels.
PyTorch provides device memory and the current HIP stream.  When the library is missing,
every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastcod.so")

OK, EINVAL, ERANGE, ENOMEM, EHIP, EBUSY, ECANCELED, ETIMEDOUT = 0, -1, -2, -3, -4, -5, -6, -7
ACCUMULATE, VALIDATE = 1, 2
VARIANT_AUTO, VARIANT_WAVE, VARIANT_STREAM = 0, 1, 2
MODE_PASSTHROUGH, MODE_END, MODE_BOTH_ENDS, MODE_SEED_END = 0, 1, 2, 3

# every symbol include/fastcod.h declares
EXPORTS = (
    "fastcod_default_opts", "fastcod_count", "fastcod_count_ex", "fastcod_volume_create",
    "fastcod_volume_bytes", "fastcod_volume_count", "fastcod_volume_destroy", "fastcod_volume_count_noalloc",
    "fastcod_validate",
    "fastcod_strerror", "fastcod_last_error", "fastcod_release",
    "fastcod_plan_create", "fastcod_plan_launch", "fastcod_plan_get_schedule", "fastcod_plan_destroy",
    "fastcod_count_batched",
    "fastcod_server_create", "fastcod_server_add_volume", "fastcod_server_submit", "fastcod_server_wait",
    "fastcod_server_cancel", "fastcod_server_get_stats", "fastcod_server_destroy",
    "fastcod_parcellate",
)
# every symbol include/fastcod_probe.h declares (ceiling probes, measurement only)
PROBE_EXPORTS = ("fastcod_probe_stream", "fastcod_probe_atomics", "fastcod_probe_lookup")
PLAN_TUNE = 1
REQ_DEVICE_POINTS, REQ_DEVICE_C, REQ_AFTER_STREAM = 1, 2, 4


class FastcodError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fastcod status {status}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_float), ("upsample", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("variant", ctypes.c_int32), ("event_begin", ctypes.c_void_p), ("event_end", ctypes.c_void_p),
                ("batch", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("pair_capacity", ctypes.c_int64)]


class Subject(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("n_streamlines", ctypes.c_int64),
                ("roi_index_vol", ctypes.c_void_p), ("target_label_vol", ctypes.c_void_p),
                ("dims", ctypes.c_int32 * 3), ("N", ctypes.c_int32), ("M", ctypes.c_int32),
                ("scale", ctypes.c_float), ("C_out", ctypes.c_void_p), ("mode", ctypes.c_int32),
                ("upsample", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("items_per_wave", ctypes.c_int32),
                ("tuned_ms", ctypes.c_float)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_uint64), ("tick_points", ctypes.c_int64), ("chunk_points", ctypes.c_int64),
                ("max_active", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("volume_id", ctypes.c_int32), ("flags", ctypes.c_uint32), ("points", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("n_streamlines", ctypes.c_int64), ("scale", ctypes.c_float),
                ("C_out", ctypes.c_void_p), ("mode", ctypes.c_int32), ("upsample", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("chunks", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("used_bytes", ctypes.c_uint64), ("pending", ctypes.c_int64),
                ("active", ctypes.c_int64), ("completed", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("volume_builds", ctypes.c_int64), ("evictions", ctypes.c_int64), ("failed", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p


def load(path: str = LIB_PATH):
    """Loads the library (once); raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FastcodError(EINVAL, f"{path} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.fastcod_default_opts.restype = Opts
    lib.fastcod_count.argtypes = [_vp, _vp, i64, _vp, _vp, _vp, i32, i32, _vp, _vp]
    lib.fastcod_count_ex.argtypes = [_vp, _vp, i64, _vp, _vp, _vp, i32, i32, _vp, ctypes.POINTER(Opts), _vp]
    lib.fastcod_volume_create.argtypes = [_vp, _vp, _vp, i32, i32, _vp, ctypes.POINTER(_vp)]
    lib.fastcod_volume_bytes.argtypes = [_vp]
    lib.fastcod_volume_bytes.restype = ctypes.c_size_t
    lib.fastcod_volume_count.argtypes = [_vp, _vp, _vp, i64, _vp, ctypes.POINTER(Opts), _vp]
    lib.fastcod_volume_destroy.argtypes = [_vp]
    lib.fastcod_volume_count_noalloc.argtypes = [_vp, _vp, _vp, i64, _vp, ctypes.POINTER(Opts), _vp]
    lib.fastcod_validate.argtypes = [_vp, i64, _vp, _vp, _vp, i32, i32, _vp]
    lib.fastcod_strerror.argtypes = [ctypes.c_int]
    lib.fastcod_strerror.restype = ctypes.c_char_p
    lib.fastcod_last_error.restype = ctypes.c_char_p
    lib.fastcod_plan_create.argtypes = [ctypes.POINTER(Subject), i32, u32, ctypes.c_char_p, _vp, ctypes.POINTER(_vp)]
    lib.fastcod_plan_launch.argtypes = [_vp, _vp]
    lib.fastcod_plan_get_schedule.argtypes = [_vp, ctypes.POINTER(Schedule)]
    lib.fastcod_plan_destroy.argtypes = [_vp]
    lib.fastcod_count_batched.argtypes = [ctypes.POINTER(Subject), i32, _vp]
    lib.fastcod_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]
    lib.fastcod_server_add_volume.argtypes = [_vp, _vp, _vp, _vp, i32, i32, ctypes.POINTER(i32)]
    lib.fastcod_server_submit.argtypes = [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.fastcod_server_wait.argtypes = [_vp, ctypes.c_uint64, i64, ctypes.POINTER(RequestInfo)]
    lib.fastcod_server_cancel.argtypes = [_vp, ctypes.c_uint64]
    lib.fastcod_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    lib.fastcod_server_destroy.argtypes = [_vp]
    lib.fastcod_parcellate.argtypes = [_vp, i32, i32, _vp, _vp, _vp, _vp]
    lib.fastcod_probe_stream.argtypes = [_vp, i64, _vp, _vp]
    lib.fastcod_probe_atomics.argtypes = [_vp, i64, _vp, i64, _vp]
    lib.fastcod_probe_lookup.argtypes = [_vp, _vp, i64, ctypes.c_float, _vp, _vp]
    for name in ("fastcod_count", "fastcod_count_ex", "fastcod_volume_create", "fastcod_volume_count",
                 "fastcod_volume_count_noalloc",
                 "fastcod_volume_destroy", "fastcod_validate", "fastcod_release", "fastcod_plan_create",
                 "fastcod_plan_launch", "fastcod_plan_get_schedule", "fastcod_plan_destroy",
                 "fastcod_count_batched", "fastcod_server_create", "fastcod_server_add_volume",
                 "fastcod_server_submit", "fastcod_server_wait", "fastcod_server_cancel",
                 "fastcod_server_get_stats", "fastcod_server_destroy", "fastcod_parcellate", *PROBE_EXPORTS):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load()
        raise FastcodError(rc, f"{lib.fastcod_strerror(rc).decode()}: {lib.fastcod_last_error().decode()}")


_dummy = {}


def _points_ptr(points: torch.Tensor) -> int:
    """Device address of the points; an empty point array gets a valid (never read) address."""
    if points.numel() > 0:
        return points.data_ptr()
    d = _dummy.get(points.device)
    if d is None:
        d = _dummy[points.device] = torch.zeros(4, dtype=torch.float32, device=points.device)
    return d.data_ptr()


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: torch.Tensor, dtype, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape[1:]) != shape:
        raise ValueError(f"{name} has shape {tuple(t.shape)}")
    return t


def make_opts(scale: float = 1.0, upsample: int = 1, accumulate: bool = False, validate: bool = False,
              variant: int = VARIANT_AUTO, events: Optional[Tuple[int, int]] = None, batch: int = 0,
              blocks_per_cu: int = 0, mode: int = MODE_PASSTHROUGH, pair_capacity: int = 0) -> Opts:
    o = load().fastcod_default_opts()
    o.scale = float(scale)
    o.upsample = int(upsample)
    o.flags = (ACCUMULATE if accumulate else 0) | (VALIDATE if validate else 0)
    o.variant = int(variant)
    if events is not None:
        o.event_begin, o.event_end = events
    o.batch = int(batch)
    o.blocks_per_cu = int(blocks_per_cu)
    o.mode = int(mode)
    o.pair_capacity = int(pair_capacity)
    return o


def count(points: torch.Tensor, offsets: torch.Tensor, roi: torch.Tensor, lab: torch.Tensor, N: int, M: int, *,
          scale: float = 1.0, upsample: int = 1, accumulate: bool = False, validate: bool = False,
          variant: int = VARIANT_AUTO, out: Optional[torch.Tensor] = None, stream=None,
          events: Optional[Tuple[int, int]] = None, batch: int = 0,
          blocks_per_cu: int = 0, mode: int = MODE_PASSTHROUGH, pair_capacity: int = 0) -> torch.Tensor:
    """C[N, M] (int32, on the points' device) of the pass-through definition (fastcod_count_ex).

    points [P,3] float32, offsets [S+1] int64, roi/lab [Z,Y,X] int32, all on one HIP device.
    Asynchronous on ``stream`` (default: the current torch stream)."""
    lib = load()
    _dev(points, torch.float32, "points", (3,))
    _dev(offsets, torch.int64, "offsets")
    _dev(roi, torch.int32, "roi")
    _dev(lab, torch.int32, "lab")
    if roi.dim() != 3 or roi.shape != lab.shape:
        raise ValueError("roi and lab must be [Z,Y,X] volumes of one shape")
    if out is None:
        out = (torch.empty if not accumulate else torch.zeros)((N, M), dtype=torch.int32, device=points.device)
    _dev(out, torch.int32, "out")
    if tuple(out.shape) != (N, M):
        raise ValueError("out must be [N, M]")
    dims = (ctypes.c_int32 * 3)(int(roi.shape[2]), int(roi.shape[1]), int(roi.shape[0]))
    o = make_opts(scale, upsample, accumulate, validate, variant, events, batch, blocks_per_cu, mode, pair_capacity)
    S = int(offsets.shape[0]) - 1
    with torch.cuda.device(points.device):
        _check(lib.fastcod_count_ex(_points_ptr(points), offsets.data_ptr(), S, roi.data_ptr(), lab.data_ptr(),
                                    dims, int(N), int(M), out.data_ptr(), ctypes.byref(o), _stream_ptr(stream)))
    return out


class Volume:
    """Resident compact volume (fastcod_volume_*): built once, counted against many times."""

    def __init__(self, roi: torch.Tensor, lab: torch.Tensor, N: int, M: int, stream=None):
        lib = load()
        _dev(roi, torch.int32, "roi")
        _dev(lab, torch.int32, "lab")
        if roi.dim() != 3 or roi.shape != lab.shape:
            raise ValueError("roi and lab must be [Z,Y,X] volumes of one shape")
        self.N, self.M = int(N), int(M)
        self.dims = (int(roi.shape[2]), int(roi.shape[1]), int(roi.shape[0]))
        self.device = roi.device
        h = _vp()
        with torch.cuda.device(roi.device):
            _check(lib.fastcod_volume_create(roi.data_ptr(), lab.data_ptr(), (ctypes.c_int32 * 3)(*self.dims),
                                             self.N, self.M, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self) -> int:
        return self._h.value

    @property
    def nbytes(self) -> int:
        return int(load().fastcod_volume_bytes(self._h))

    def count(self, points: torch.Tensor, offsets: torch.Tensor, *, scale: float = 1.0, upsample: int = 1,
              accumulate: bool = False, out: Optional[torch.Tensor] = None, stream=None, events=None,
              mode: int = MODE_PASSTHROUGH, pair_capacity: int = 0, batch: int = 0, blocks_per_cu: int = 0,
              noalloc: bool = False) -> torch.Tensor:
        """C of these streamlines against the resident volume (fastcod_volume_count, or with
        ``noalloc`` fastcod_volume_count_noalloc: the library's fixed scratch area, no allocation;
        then ``out`` must be given so that nothing is allocated here either)."""
        lib = load()
        _dev(points, torch.float32, "points", (3,))
        _dev(offsets, torch.int64, "offsets")
        if out is None:
            if noalloc:
                raise ValueError("noalloc counts need a preallocated out")
            out = (torch.empty if not accumulate else torch.zeros)((self.N, self.M), dtype=torch.int32,
                                                                  device=points.device)
        _dev(out, torch.int32, "out")
        if tuple(out.shape) != (self.N, self.M):
            raise ValueError(f"out must be [{self.N}, {self.M}]")
        o = make_opts(scale, upsample, accumulate, False, VARIANT_STREAM, events, batch, blocks_per_cu, mode,
                      pair_capacity)
        fn = lib.fastcod_volume_count_noalloc if noalloc else lib.fastcod_volume_count
        with torch.cuda.device(points.device):
            _check(fn(self._h, _points_ptr(points), offsets.data_ptr(), int(offsets.shape[0]) - 1, out.data_ptr(),
                      ctypes.byref(o), _stream_ptr(stream)))
        return out

    def close(self):
        if self._h is not None and self._h.value:
            _check(load().fastcod_volume_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def parcellate(C: torch.Tensor, labels: bool = True, fractions: bool = True, sums: bool = True, stream=None,
               events=None):
    """Parcellation outputs of C [N, M] int32 (fastcod_parcellate): (label [N] int32, frac [N, M]
    float32, sums [N] int64), each None when not asked for.  ``events`` = (begin, end) hipEvents
    recorded around the launch on ``stream``."""
    lib = load()
    _dev(C, torch.int32, "C")
    if C.dim() != 2:
        raise ValueError("C must be [N, M]")
    N, M = int(C.shape[0]), int(C.shape[1])
    lab = torch.empty(N, dtype=torch.int32, device=C.device) if labels else None
    frac = torch.empty((N, M), dtype=torch.float32, device=C.device) if fractions else None
    sm = torch.empty(N, dtype=torch.int64, device=C.device) if sums else None
    ptr = lambda t: t.data_ptr() if t is not None and t.numel() else None   # noqa: E731
    with torch.cuda.device(C.device):
        st = _stream_ptr(stream)
        hip = None
        if events is not None:
            hip = ctypes.CDLL("libamdhip64.so")
            hip.hipEventRecord.argtypes = [_vp, _vp]
            hip.hipEventRecord(events[0], st)
        _check(lib.fastcod_parcellate(ptr(C), N, M, ptr(lab), ptr(frac), ptr(sm), st))
        if hip is not None:
            hip.hipEventRecord(events[1], st)
    return lab, frac, sm


def validate(offsets: torch.Tensor, roi: torch.Tensor, lab: torch.Tensor, N: int, M: int, stream=None) -> None:
    """Raises FastcodError(ERANGE) when offsets are malformed or volume values exceed N / M."""
    lib = load()
    dims = (ctypes.c_int32 * 3)(int(roi.shape[2]), int(roi.shape[1]), int(roi.shape[0]))
    with torch.cuda.device(roi.device):
        _check(lib.fastcod_validate(offsets.data_ptr(), int(offsets.shape[0]) - 1, roi.data_ptr(), lab.data_ptr(),
                                    dims, int(N), int(M), _stream_ptr(stream)))


def release() -> None:
    _check(load().fastcod_release())


def make_subject(points: torch.Tensor, offsets: torch.Tensor, roi: torch.Tensor, lab: torch.Tensor, N: int, M: int,
                 C: torch.Tensor, scale: float = 1.0, mode: int = MODE_PASSTHROUGH, upsample: int = 1) -> Subject:
    """C-ABI descriptor of one subject of a batched plan (the tensors must outlive the plan)."""
    _dev(points, torch.float32, "points", (3,))
    _dev(offsets, torch.int64, "offsets")
    _dev(roi, torch.int32, "roi")
    _dev(lab, torch.int32, "lab")
    _dev(C, torch.int32, "C")
    if roi.dim() != 3 or roi.shape != lab.shape or tuple(C.shape) != (N, M):
        raise ValueError("bad volume or C shape")
    u = Subject()
    u.points = _points_ptr(points)
    u.offsets = offsets.data_ptr()
    u.n_streamlines = int(offsets.shape[0]) - 1
    u.roi_index_vol = roi.data_ptr()
    u.target_label_vol = lab.data_ptr()
    u.dims[0], u.dims[1], u.dims[2] = int(roi.shape[2]), int(roi.shape[1]), int(roi.shape[0])
    u.N, u.M = int(N), int(M)
    u.scale = float(scale)
    u.C_out = C.data_ptr()
    u.mode = int(mode)
    u.upsample = int(upsample)
    return u


class Plan:
    """Batched counting plan (fastcod_plan_*): one captured graph counting every subject.

    ``subjects``: sequence of dicts with points, offsets, roi, lab, N, M, C and optional scale, mode
    and upsample (CUDA tensors, kept alive by the plan object)."""

    def __init__(self, subjects, tune: bool = False, tune_cache: Optional[str] = None, stream=None):
        lib = load()
        self._keep = list(subjects)
        arr = (Subject * len(subjects))(*[make_subject(d["points"], d["offsets"], d["roi"], d["lab"], d["N"], d["M"],
                                                       d["C"], d.get("scale", 1.0), d.get("mode", 0),
                                                       d.get("upsample", 1)) for d in subjects])
        h = _vp()
        dev = subjects[0]["points"].device
        with torch.cuda.device(dev):
            _check(lib.fastcod_plan_create(arr, len(subjects), PLAN_TUNE if tune else 0,
                                           tune_cache.encode() if tune_cache else None, _stream_ptr(stream),
                                           ctypes.byref(h)))
        self._h = h
        self.device = dev

    def launch(self, stream=None) -> None:
        with torch.cuda.device(self.device):
            _check(load().fastcod_plan_launch(self._h, _stream_ptr(stream)))

    @property
    def schedule(self) -> dict:
        sc = Schedule()
        _check(load().fastcod_plan_get_schedule(self._h, ctypes.byref(sc)))
        return {"batch": sc.batch, "blocks_per_cu": sc.blocks_per_cu, "items_per_wave": sc.items_per_wave,
                "tuned_ms": sc.tuned_ms}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(load().fastcod_plan_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def count_batched(subjects, stream=None) -> None:
    """One-shot batched count (fastcod_count_batched): every subject's C is overwritten."""
    lib = load()
    arr = (Subject * len(subjects))(*[make_subject(d["points"], d["offsets"], d["roi"], d["lab"], d["N"], d["M"],
                                                   d["C"], d.get("scale", 1.0), d.get("mode", 0), d.get("upsample", 1))
                                      for d in subjects])
    with torch.cuda.device(subjects[0]["points"].device):
        _check(lib.fastcod_count_batched(arr, len(subjects), _stream_ptr(stream)))


class Server:
    """Request server (fastcod_server_*) on the current device.

    Volumes are registered from host arrays; requests bring points (host or device tensor),
    host int64 offsets and a C destination (host or device int32 [N, M]).  The server keeps a
    reference to every submitted array until the request has been waited for.  Host arrays
    should be pinned (``torch.empty(..., pin_memory=True)``) for the copies to overlap."""

    def __init__(self, memory_budget: int = 0, tick_points: int = 0, chunk_points: int = 0, max_active: int = 0):
        lib = load()
        cfg = ServerConfig(int(memory_budget), int(tick_points), int(chunk_points), int(max_active), 0)
        h = _vp()
        _check(lib.fastcod_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}
        self._vols = {}

    def add_volume(self, roi, lab, N: int, M: int) -> int:
        """Registers a [Z,Y,X] int32 volume pair (numpy arrays or CPU tensors); returns its id."""
        roi = _host_i32(roi, "roi")
        lab = _host_i32(lab, "lab")
        if roi.dim() != 3 or roi.shape != lab.shape:
            raise ValueError("roi and lab must be [Z,Y,X] volumes of one shape")
        dims = (ctypes.c_int32 * 3)(int(roi.shape[2]), int(roi.shape[1]), int(roi.shape[0]))
        vid = ctypes.c_int32()
        _check(load().fastcod_server_add_volume(self._h, roi.data_ptr(), lab.data_ptr(), dims, int(N), int(M),
                                                ctypes.byref(vid)))
        self._vols[vid.value] = (int(N), int(M))
        return vid.value

    def submit(self, volume_id: int, points: torch.Tensor, offsets, out: torch.Tensor, scale: float = 1.0,
               mode: int = MODE_PASSTHROUGH, upsample: int = 1, stream=None) -> int:
        """Queues a request; ``out`` ([N, M] int32, host or device) receives C.  Returns its id.

        When points or out are device tensors, the server orders its accesses to them after the
        work enqueued so far on ``stream`` (default: the current torch stream)."""
        if not isinstance(points, torch.Tensor) or points.dtype != torch.float32 or not points.is_contiguous() \
                or points.dim() != 2 or points.shape[1] != 3:
            raise TypeError("points must be a contiguous float32 [P, 3] tensor")
        offsets = _host_i64(offsets, "offsets")
        if not isinstance(out, torch.Tensor) or out.dtype != torch.int32 or not out.is_contiguous():
            raise TypeError("out must be a contiguous int32 tensor")
        N, M = self._vols.get(volume_id, (None, None))
        if N is not None and tuple(out.shape) != (N, M):
            raise ValueError(f"out must be [{N}, {M}]")
        flags = (REQ_DEVICE_POINTS if points.is_cuda else 0) | (REQ_DEVICE_C if out.is_cuda else 0)
        st = None
        if points.is_cuda or out.is_cuda:
            flags |= REQ_AFTER_STREAM
            st = _stream_ptr(stream)
        pts_ptr = _points_ptr(points) if points.is_cuda else (points.data_ptr() if points.numel() else None)
        r = Request(int(volume_id), flags, pts_ptr, offsets.data_ptr(), int(offsets.shape[0]) - 1, float(scale),
                    out.data_ptr(), int(mode), int(upsample), st)
        rid = ctypes.c_uint64()
        _check(load().fastcod_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._keep[rid.value] = (points, offsets, out)
        return rid.value

    def wait(self, request_id: int, timeout: Optional[float] = None) -> dict:
        """Waits for a request; returns its info dict (``status`` 0 = C written).  Raises
        FastcodError(ETIMEDOUT) if it is still running after ``timeout`` seconds."""
        info = RequestInfo()
        us = -1 if timeout is None else int(timeout * 1e6)
        rc = load().fastcod_server_wait(self._h, int(request_id), us, ctypes.byref(info))
        if rc in (ETIMEDOUT, EINVAL):
            _check(rc)
        self._keep.pop(int(request_id), None)
        return {"status": rc, "t_submit_ns": info.t_submit_ns, "t_admit_ns": info.t_admit_ns,
                "t_done_ns": info.t_done_ns, "chunks": info.chunks, "device_bytes": info.device_bytes}

    def cancel(self, request_id: int) -> None:
        _check(load().fastcod_server_cancel(self._h, int(request_id)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().fastcod_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_ if k != "reserved"}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(load().fastcod_server_destroy(self._h))
        self._h = None
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_i32(a, name):
    t = torch.as_tensor(a)
    if t.is_cuda or t.dtype != torch.int32:
        raise TypeError(f"{name} must be a host int32 array")
    return t.contiguous()


def _host_i64(a, name):
    t = torch.as_tensor(a)
    if t.is_cuda or t.dtype != torch.int64 or t.dim() != 1 or t.shape[0] < 1:
        raise TypeError(f"{name} must be a host int64 [S+1] array")
    return t.contiguous()


# ---- ceiling probes (include/fastcod_probe.h): each enqueues one kernel on the stream ----

def _sink(device):
    d = _dummy.get(("sink", device))
    if d is None:
        d = _dummy[("sink", device)] = torch.zeros(1, dtype=torch.int32, device=device)
    return d.data_ptr()


def probe_stream(points: torch.Tensor, stream=None) -> None:
    """Reads every point once (12 bytes each) with the counting kernel's access pattern."""
    _dev(points, torch.float32, "points", (3,))
    with torch.cuda.device(points.device):
        _check(load().fastcod_probe_stream(_points_ptr(points), int(points.shape[0]), _sink(points.device),
                                           _stream_ptr(stream)))


def probe_atomics(target: torch.Tensor, idx: torch.Tensor, stream=None) -> None:
    """target[idx[k]] += 1 with no-return device atomics (int32 target, int32/uint32 indices)."""
    _dev(target, torch.int32, "target")
    if not isinstance(idx, torch.Tensor) or not idx.is_cuda or idx.dtype != torch.int32 or not idx.is_contiguous():
        raise TypeError("idx must be a contiguous int32 CUDA tensor (read as uint32)")
    with torch.cuda.device(target.device):
        _check(load().fastcod_probe_atomics(target.data_ptr(), int(target.numel()), idx.data_ptr(), int(idx.numel()),
                                            _stream_ptr(stream)))


def probe_lookup(vol: "Volume", points: torch.Tensor, scale: float = 1.0, stream=None) -> None:
    """The point stream plus every point's lookups in the resident volume (no de-duplication, no C)."""
    _dev(points, torch.float32, "points", (3,))
    with torch.cuda.device(points.device):
        _check(load().fastcod_probe_lookup(vol.handle, _points_ptr(points), int(points.shape[0]), float(scale),
                                           _sink(points.device), _stream_ptr(stream)))
