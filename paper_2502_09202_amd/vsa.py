"""Python binding of libvsa (argument marshalling only).

Every function here forwards to the C ABI of the same name in
``include/vsa.h`` (``vsa_<name>``).  All computation runs in the library's
HIP kernels; if the library is missing this module raises instead of falling
back to anything else.  PyTorch is optional: device planes can be handed over
as raw device pointers, or as CUDA tensors through :func:`stream_push_tensor`.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvsa.so")
DEFAULT_PARAMS_JSON = os.path.join(HERE, "params", "default.json")

OK, E_INVAL, E_NOMEM, E_ADMIT, E_STATE, E_DEVICE, E_AGAIN, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
SCHEDULE_SPARSE, SCHEDULE_DENSE = 0, 1
SRC_HOST, SRC_DEVICE_COPY, SRC_DEVICE_BORROW, SRC_HOST_BORROW = 0, 1, 2, 3
F_HAS_PAIR, F_STATIC, F_FAST_FIRED, F_IN_TRANSITION = 1, 2, 4, 8
F_KEYFRAME, F_SHOT_START, F_ANALYZED = 16, 32, 64
SAMPLING_NAMES = {0: "undetermined", 1: "progressive", 2: "tff", 3: "bff", 4: "pulldown32"}


class VsaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vsa error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("block", C.c_int32), ("radius", C.c_int32), ("wmax", C.c_int32),
        ("lf_offset", C.c_int32), ("k_max", C.c_int32), ("a_static_fx", C.c_int32),
        ("w_hist", C.c_int32), ("n_ss", C.c_int32),
        ("a0", C.c_double), ("rho_f", C.c_double), ("theta_f", C.c_double), ("theta_f0", C.c_double),
        ("rho_d", C.c_double), ("theta_d", C.c_double), ("gamma", C.c_double),
        ("tau_c", C.c_double), ("eps", C.c_double), ("tau_p", C.c_double),
        ("theta_kf", C.c_double), ("search", C.c_int32), ("refine", C.c_int32),
    ]


class EngineConfig(C.Structure):
    _fields_ = [
        ("device", C.c_int32), ("max_streams", C.c_int32), ("hbm_budget_bytes", C.c_uint64),
        ("schedule", C.c_int32), ("use_graph", C.c_int32), ("params", C.POINTER(Params)),
        ("debug_log", C.c_int32), ("me_wgs_per_cu", C.c_int32), ("profile", C.c_int32),
        ("no_intensity", C.c_int32), ("profile_every", C.c_int32), ("params_json", C.c_char_p),
        ("autotune_cache", C.c_char_p),
    ]


class ClipConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("bit_depth", C.c_int32),
                ("k_max", C.c_int32), ("chunk", C.c_int32), ("schedule", C.c_int32), ("no_intensity", C.c_int32),
                ("me_wgs_per_cu", C.c_int32), ("params", C.POINTER(Params)), ("debug_log", C.c_int32)]


class StreamDesc(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("bit_depth", C.c_int32),
                ("fps_num", C.c_int32), ("fps_den", C.c_int32), ("k_max", C.c_int32)]


FRAME_DTYPE = np.dtype([
    ("frame", "<i8"), ("pts", "<i8"), ("flags", "<i4"), ("shot_id", "<i4"), ("boundary", "<i4"),
    ("boundary_k", "<i4"), ("ncc", "<f8"), ("swr", "<f8"), ("amm", "<f8"), ("act", "<f8"),
    ("mom", "<i8", (5,)), ("n_pix", "<i8"), ("amm_num", "<i8"), ("n_blocks", "<i4"),
    ("field_mask", "<u4"), ("v", "<f8", (3,)), ("h_mean", "<f8"), ("h_std", "<f8"), ("h_mad", "<f8"),
])
SHOT_DTYPE = np.dtype([
    ("shot_id", "<i4"), ("pad0", "<i4"), ("first", "<i8"), ("last", "<i8"),
    ("in_boundary", "<i4"), ("in_k", "<i4"), ("sampling", "<i4"), ("pulldown_phase", "<i4"),
    ("n_analyzed", "<i4"), ("final", "<i4"),
])
KEY_DTYPE = np.dtype([("kind", "<i4"), ("ref", "<i4"), ("oth", "<i4"), ("ref_field", "<i4"),
                      ("oth_field", "<i4"), ("level", "<i4")])

# every symbol the header declares
SYMBOLS = [
    "vsa_abi_version", "vsa_default_params", "vsa_engine_create", "vsa_engine_destroy",
    "vsa_stream_footprint", "vsa_stream_open", "vsa_stream_push", "vsa_stream_end",
    "vsa_stream_done", "vsa_step", "vsa_sync", "vsa_poll_frames", "vsa_poll_shots",
    "vsa_get_motion", "vsa_stream_close", "vsa_engine_counters", "vsa_engine_tuning", "vsa_get_histogram", "vsa_last_error",
    "vsa_debug_levels", "vsa_debug_pair", "vsa_debug_finish", "vsa_debug_decide",
    "vsa_flow_scratch_bytes", "vsa_flow_pair", "vsa_debug_flow_pair", "vsa_params_from_json",
    "vsa_debug_measure_log", "vsa_stream_push_batch", "vsa_engine_kernel_times", "vsa_collect",
    "vsa_poll_frames_all", "vsa_clip_create", "vsa_clip_destroy", "vsa_clip_run", "vsa_clip_counters", "vsa_clip_debug_log",
    "vsa_debug_clip_chunks", "vsa_pair_noalloc",
]

_lib = None


def lib():
    """Load libvsa.so (built in-tree by paper_2502_09202_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2502_09202_amd/build.py")
    # PyTorch ships its own HIP runtime under the same soname.  Loading it first
    # makes libvsa bind to that one, so a process that also uses torch (for
    # device buffers and streams) holds a single HIP runtime; loaded the other
    # way round, torch would bring a second runtime that then finds no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, i64, u64 = C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "vsa_abi_version": (i32, []),
        "vsa_default_params": (None, [C.POINTER(Params)]),
        "vsa_engine_create": (i32, [C.POINTER(EngineConfig), C.POINTER(P)]),
        "vsa_engine_destroy": (None, [P]),
        "vsa_stream_footprint": (u64, [P, C.POINTER(StreamDesc)]),
        "vsa_stream_open": (i32, [P, C.POINTER(StreamDesc), C.POINTER(i32)]),
        "vsa_stream_push": (i32, [P, i32, P, i64, i32, i64]),
        "vsa_stream_end": (i32, [P, i32]),
        "vsa_stream_done": (i32, [P, i32]),
        "vsa_step": (i32, [P, P]),
        "vsa_sync": (i32, [P]),
        "vsa_collect": (i32, [P, C.POINTER(i64)]),
        "vsa_poll_frames": (i32, [P, i32, P, i32]),
        "vsa_poll_shots": (i32, [P, i32, P, i32]),
        "vsa_poll_frames_all": (i32, [P, P, P, i32]),
        "vsa_get_motion": (i32, [P, i32, i64, P, i32, C.POINTER(i32), C.POINTER(i32)]),
        "vsa_stream_close": (i32, [P, i32]),
        "vsa_engine_counters": (i32, [P, P, i32]),
        "vsa_last_error": (C.c_char_p, []),
        "vsa_debug_levels": (i32, [C.POINTER(Params), P, i32, i32, i64, i32, P, i64, C.POINTER(i64)]),
        "vsa_debug_pair": (i32, [C.POINTER(Params), P, P, i32, i32, i32, i32, P, P, P, P]),
        "vsa_flow_scratch_bytes": (i64, [i32, i32]),
        "vsa_params_from_json": (i32, [C.c_char_p, C.POINTER(Params)]),
        "vsa_flow_pair": (i32, [C.POINTER(Params), P, P, i32, i32, i64, i32, P, i64, P, P, P]),
        "vsa_debug_flow_pair": (i32, [C.POINTER(Params), P, P, i32, i32, i32, P, P, P]),
        "vsa_debug_finish": (i32, [P, i64, C.c_double, P]),
        "vsa_debug_decide": (i32, [C.POINTER(Params), i32, i32, i32, P, P, P, P, P, P, P, P, P, i32,
                                   C.POINTER(i32), P, i32, C.POINTER(i32)]),
        "vsa_debug_measure_log": (i32, [P, i32, P, i32]),
        "vsa_stream_push_batch": (i32, [P, i32, P, P, P, i32, P, P]),
        "vsa_engine_kernel_times": (i32, [P, P, P, i32]),
        "vsa_engine_tuning": (i32, [P, i32, P, P, P, P, i32]),
        "vsa_get_histogram": (i32, [P, i32, i64, P, i32, P]),
        "vsa_clip_create": (i32, [C.POINTER(ClipConfig), C.POINTER(P)]),
        "vsa_clip_destroy": (None, [P]),
        "vsa_clip_run": (i32, [P, P, i64, i64, i32, i32, P, P, i32, C.POINTER(i32)]),
        "vsa_clip_counters": (i32, [P, P, i32]),
        "vsa_clip_debug_log": (i32, [P, P, i32]),
        "vsa_debug_clip_chunks": (i32, [i32, i32, P, P, i32]),
        "vsa_pair_noalloc": (i32, [C.POINTER(Params), P, P, i32, i32, i64, i32, i32, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().vsa_last_error().decode(errors="replace")


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise VsaError(rc, f"{what}: {last_error()}")
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def abi_version() -> int:
    return lib().vsa_abi_version()


def default_params() -> dict:
    p = Params()
    lib().vsa_default_params(C.byref(p))
    return {k: getattr(p, k) for k, _ in Params._fields_}


def load_params(path: Optional[str] = None) -> dict:
    with open(path or DEFAULT_PARAMS_JSON) as f:
        return json.load(f)


def make_params(d: Optional[dict]) -> Params:
    p = Params()
    lib().vsa_default_params(C.byref(p))
    for k, v in (d or {}).items():
        setattr(p, k, v)
    return p


class Engine:
    """An engine handle; see vsa_engine_create."""

    def __init__(self, device: int = 0, max_streams: int = 64, hbm_budget_bytes: int = 0,
                 schedule: int = SCHEDULE_SPARSE, use_graph: int = 0, params: Optional[dict] = None,
                 debug_log: int = 0, profile: int = 0, me_wgs_per_cu: int = 0, no_intensity: int = 0,
                 profile_every: int = 0, params_json: Optional[str] = None,
                 autotune_cache: Optional[str] = None):
        self._params = make_params(params)
        self._json = None if params_json is None else params_json.encode()
        self._cache = None if autotune_cache is None else os.fsencode(autotune_cache)
        cfg = EngineConfig(device=device, max_streams=max_streams, hbm_budget_bytes=hbm_budget_bytes,
                           schedule=schedule, use_graph=use_graph,
                           params=C.pointer(self._params), debug_log=debug_log, me_wgs_per_cu=me_wgs_per_cu,
                           profile=profile, no_intensity=no_intensity, profile_every=profile_every,
                           params_json=self._json, autotune_cache=self._cache)
        h = C.c_void_p()
        _check(lib().vsa_engine_create(C.byref(cfg), C.byref(h)), "engine_create")
        self.h = h

    def close(self):
        if self.h:
            lib().vsa_engine_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- streams
    def footprint(self, width, height, bit_depth=8, k_max=0, fps=(25, 1)) -> int:
        d = StreamDesc(width, height, bit_depth, fps[0], fps[1], k_max)
        return int(lib().vsa_stream_footprint(self.h, C.byref(d)))

    def stream_open(self, width, height, bit_depth=8, k_max=0, fps=(25, 1)) -> int:
        d = StreamDesc(width, height, bit_depth, fps[0], fps[1], k_max)
        sid = C.c_int32(-1)
        _check(lib().vsa_stream_open(self.h, C.byref(d), C.byref(sid)), "stream_open")
        return sid.value

    def stream_push(self, sid: int, plane, pts: int = 0) -> int:
        """Push a host numpy plane (uint8 / uint16), copied before return."""
        a = np.ascontiguousarray(plane)
        return lib().vsa_stream_push(self.h, sid, _ptr(a), a.strides[0], SRC_HOST, pts)

    def stream_push_device(self, sid: int, dev_ptr: int, pitch_bytes: int, mode: int = SRC_DEVICE_BORROW,
                           pts: int = 0) -> int:
        return lib().vsa_stream_push(self.h, sid, C.c_void_p(dev_ptr), pitch_bytes, mode, pts)

    def stream_push_tensor(self, sid: int, t, mode: int = SRC_DEVICE_BORROW, pts: int = 0) -> int:
        """Push a 2-D CUDA tensor (uint8 / int16 / uint16 samples) by device pointer."""
        assert t.dim() == 2 and t.is_cuda and t.stride(1) == 1
        return self.stream_push_device(sid, t.data_ptr(), t.stride(0) * t.element_size(), mode, pts)

    def stream_push_batch(self, sids: np.ndarray, ptrs: np.ndarray, pitches: np.ndarray,
                          mode: int = SRC_DEVICE_BORROW, pts: Optional[np.ndarray] = None) -> int:
        """One call for many streams: sids int32[n], ptrs uint64[n] (host or device
        addresses per mode), pitches int64[n] bytes, pts int64[n] (optional)."""
        n = len(sids)
        return lib().vsa_stream_push_batch(self.h, n, _ptr(sids), _ptr(ptrs), _ptr(pitches), mode,
                                           _ptr(pts), None)

    def kernel_times(self, reset: bool = False) -> dict:
        ms = np.zeros(6, np.float64)
        n = np.zeros(6, np.uint64)
        _check(lib().vsa_engine_kernel_times(self.h, _ptr(ms), _ptr(n), int(reset)), "engine_kernel_times")
        names = ("pyramid", "me8", "me10", "me_sparse", "decide", "step")
        return {k: (float(m), int(c)) for k, m, c in zip(names, ms, n)}

    def stream_end(self, sid: int):
        _check(lib().vsa_stream_end(self.h, sid), "stream_end")

    def stream_done(self, sid: int) -> bool:
        return bool(_check(lib().vsa_stream_done(self.h, sid), "stream_done"))

    def stream_close(self, sid: int):
        _check(lib().vsa_stream_close(self.h, sid), "stream_close")

    # -- steps
    def step(self, hip_stream: Optional[int] = None):
        _check(lib().vsa_step(self.h, C.c_void_p(hip_stream) if hip_stream else None), "step")

    def sync(self):
        _check(lib().vsa_sync(self.h), "sync")

    def collect(self) -> int:
        """Publish the records of the steps the device has completed, without
        waiting; returns the number of published steps."""
        n = C.c_int64(0)
        _check(lib().vsa_collect(self.h, C.byref(n)), "collect")
        return n.value

    def poll_frames(self, sid: int, cap: int = 4096) -> np.ndarray:
        out = np.zeros(cap, FRAME_DTYPE)
        n = _check(lib().vsa_poll_frames(self.h, sid, _ptr(out), cap), "poll_frames")
        return out[:n].copy()

    def poll_frames_all(self, cap: int = 4096):
        """Records of every stream: (sids int32[n], records FRAME_DTYPE[n]), at
        most cap per call (the receive buffers are reused between calls)."""
        buf = getattr(self, "_poll_buf", None)
        if buf is None or buf[0].size < cap:
            buf = (np.zeros(cap, np.int32), np.zeros(cap, FRAME_DTYPE))
            self._poll_buf = buf
        sids, out = buf
        n = _check(lib().vsa_poll_frames_all(self.h, _ptr(sids), _ptr(out), cap), "poll_frames_all")
        return sids[:n].copy(), out[:n].copy()

    def poll_shots(self, sid: int, cap: int = 1024) -> np.ndarray:
        out = np.zeros(cap, SHOT_DTYPE)
        n = _check(lib().vsa_poll_shots(self.h, sid, _ptr(out), cap), "poll_shots")
        return out[:n].copy()

    def get_motion(self, sid: int, frame: int) -> np.ndarray:
        nbx, nby = C.c_int32(0), C.c_int32(0)
        _check(lib().vsa_get_motion(self.h, sid, frame, None, 0, C.byref(nbx), C.byref(nby)), "get_motion")
        mv = np.zeros((nby.value, nbx.value, 2), np.int8)
        _check(lib().vsa_get_motion(self.h, sid, frame, _ptr(mv), nbx.value * nby.value,
                                    C.byref(nbx), C.byref(nby)), "get_motion")
        return mv

    def counters(self) -> dict:
        out = np.zeros(14, np.uint64)
        _check(lib().vsa_engine_counters(self.h, _ptr(out), 14), "engine_counters")
        keys = ("steps", "streams_open", "admitted", "refused", "bytes_in_use", "budget",
                "sparse_tasks", "consecutive_tasks", "consecutive_blocks", "sparse_blocks",
                "host_ns_build", "host_ns_upload", "host_ns_launch", "host_ns_step")
        return {k: int(v) for k, v in zip(keys, out)}

    def histogram(self, sid: int, frame: int) -> np.ndarray:
        """Intensity histogram H(t) of a frame still held on the device
        (working-level image, 2^bit_depth bins)."""
        nb = C.c_int32(0)
        _check(lib().vsa_get_histogram(self.h, sid, frame, None, 0, C.byref(nb)), "get_histogram")
        out = np.zeros(nb.value, np.uint32)
        _check(lib().vsa_get_histogram(self.h, sid, frame, _ptr(out), nb.value, C.byref(nb)), "get_histogram")
        return out

    def tuning(self) -> dict:
        """Launch autotuner state per size bucket that has timings: the chosen
        candidate (-1 while tuning) and each candidate's grids, windows and
        step period in ms (fastest window)."""
        out = {}
        for bucket in range(32):
            best = C.c_int32(-1)
            wgs = np.zeros((8, 2), np.int32)
            win = np.zeros(8, np.int32)
            ms = np.zeros(8, np.float64)
            n = _check(lib().vsa_engine_tuning(self.h, bucket, C.byref(best), _ptr(wgs), _ptr(win), _ptr(ms), 8),
                       "engine_tuning")
            if best.value >= 0 or win[:n].any():
                out[bucket] = {"best": best.value,
                               "candidates": [{"wgs": tuple(int(x) for x in wgs[c]), "windows": int(win[c]),
                                               "step_ms": round(float(ms[c]), 4)} for c in range(n)]}
        return out

    def measure_log(self, sid: int) -> np.ndarray:
        n = _check(lib().vsa_debug_measure_log(self.h, sid, None, 0), "debug_measure_log")
        out = np.zeros(max(n, 1), KEY_DTYPE)
        _check(lib().vsa_debug_measure_log(self.h, sid, _ptr(out), n), "debug_measure_log")
        return out[:n].copy()


class Clip:
    """An offline clip analyser; see vsa_clip_create (one clip at a time, all
    its frames at hand, processed `chunk` frames per launch)."""

    def __init__(self, width: int, height: int, bit_depth: int = 8, k_max: int = 0, chunk: int = 0,
                 dense: bool = False, params: Optional[dict] = None, no_intensity: int = 0,
                 me_wgs_per_cu: int = 0, device: int = 0, debug_log: bool = False):
        self._params = make_params(params)
        cfg = ClipConfig(device=device, width=width, height=height, bit_depth=bit_depth, k_max=k_max, chunk=chunk,
                         schedule=SCHEDULE_DENSE if dense else SCHEDULE_SPARSE, no_intensity=no_intensity,
                         me_wgs_per_cu=me_wgs_per_cu, params=C.pointer(self._params), debug_log=int(debug_log))
        h = C.c_void_p()
        _check(lib().vsa_clip_create(C.byref(cfg), C.byref(h)), "clip_create")
        self.h = h
        self.shape = (height, width)
        self.bit_depth = bit_depth

    def close(self):
        if self.h:
            lib().vsa_clip_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _run(self, ptr, stride, pitch, T, src):
        recs = np.zeros(T, FRAME_DTYPE)
        shots = np.zeros(T + 1, SHOT_DTYPE)
        ns = C.c_int32(0)
        _check(lib().vsa_clip_run(self.h, ptr, stride, pitch, T, src, _ptr(recs), _ptr(shots), shots.size,
                                  C.byref(ns)), "clip_run")
        return {"frames": recs, "shots": shots[:ns.value].copy()}

    def run(self, frames: np.ndarray) -> dict:
        """Analyse a host clip [T, H, W] (uint8, or uint16 for 10 bits)."""
        a = np.ascontiguousarray(frames)
        assert a.ndim == 3 and a.shape[1:] == self.shape
        pitch = a.shape[2] * a.itemsize          # (an empty array's strides may read 0)
        return self._run(_ptr(a), pitch * a.shape[1], pitch, a.shape[0], SRC_HOST)

    def run_tensor(self, t) -> dict:
        """Analyse a CUDA tensor [T, H, W] read in place (rows contiguous)."""
        assert t.dim() == 3 and t.is_cuda and t.stride(2) == 1 and tuple(t.shape[1:]) == self.shape
        es = t.element_size()
        return self._run(C.c_void_p(t.data_ptr()), t.stride(0) * es, t.stride(1) * es, t.shape[0],
                         SRC_DEVICE_BORROW)

    def counters(self) -> dict:
        out = np.zeros(6, np.uint64)
        _check(lib().vsa_clip_counters(self.h, _ptr(out), 6), "clip_counters")
        return dict(zip(("chunks", "decision_launches", "waits", "sparse_tasks", "speculative_tasks",
                         "requested_measures"), (int(x) for x in out)))

    def measure_log(self) -> np.ndarray:
        """[n, 6] int32 (kind, ref, oth, ref_field, oth_field, level) of the sparse
        measures the sequential pass requested in the last run (debug_log)."""
        n = _check(lib().vsa_clip_debug_log(self.h, None, 0), "clip_debug_log")
        out = np.zeros((max(n, 1), 6), np.int32)
        _check(lib().vsa_clip_debug_log(self.h, _ptr(out), n), "clip_debug_log")
        return out[:n].copy()


def run_clip(frames: np.ndarray, params: Optional[dict] = None, bit_depth: int = 8, dense: bool = False,
             k_max: int = 0, device: int = 0, debug_log: bool = False, want_mv: bool = False, **engine_kw):
    """Push a whole host clip [T, H, W] through one stream; returns records and shots."""
    T, H, W = frames.shape
    with Engine(device=device, max_streams=1, params=params,
                schedule=SCHEDULE_DENSE if dense else SCHEDULE_SPARSE, debug_log=int(debug_log), **engine_kw) as e:
        sid = e.stream_open(W, H, bit_depth, k_max)
        recs, shots, mvs = [], [], []
        for t in range(T):
            _check(e.stream_push(sid, frames[t], pts=t), "stream_push")
            if t == T - 1:
                e.stream_end(sid)
            e.step()
            if want_mv and t >= 1:
                e.sync()
                mvs.append(e.get_motion(sid, t - 1))
        guard = 0
        while not e.stream_done(sid):
            e.step()
            e.sync()
            guard += 1
            if guard > 4 * (T + 64):
                raise VsaError(E_STATE, "stream did not finish")
        e.sync()
        recs.append(e.poll_frames(sid, T + 16))
        shots.append(e.poll_shots(sid, T + 16))
        out = {"frames": np.concatenate(recs), "shots": np.concatenate(shots)}
        if debug_log:
            out["keys"] = e.measure_log(sid)
        if want_mv:
            out["mv"] = np.stack(mvs) if mvs else np.zeros((0,), np.int8)
        return out


# -- test hooks ---------------------------------------------------------------

def debug_clip_chunks(chunk: int, n_frames: int):
    """(starts, counts) of the chunks vsa_clip_run takes an n_frames clip in."""
    n = _check(lib().vsa_debug_clip_chunks(chunk, n_frames, None, None, 0), "debug_clip_chunks")
    starts, counts = np.zeros(n, np.int32), np.zeros(n, np.int32)
    _check(lib().vsa_debug_clip_chunks(chunk, n_frames, _ptr(starts), _ptr(counts), n), "debug_clip_chunks")
    return starts, counts


def debug_levels(plane: np.ndarray, params: Optional[dict] = None, bit_depth: int = 8) -> np.ndarray:
    a = np.ascontiguousarray(plane)
    H, W = a.shape
    p = make_params(params)
    n = C.c_int64(0)
    _check(lib().vsa_debug_levels(C.byref(p), _ptr(a), W, H, a.strides[0], bit_depth, None, 0, C.byref(n)),
           "debug_levels")
    out = np.zeros(n.value, np.uint16)
    _check(lib().vsa_debug_levels(C.byref(p), _ptr(a), W, H, a.strides[0], bit_depth, _ptr(out), out.size,
                                  C.byref(n)), "debug_levels")
    return out


def debug_pair(I: np.ndarray, J: np.ndarray, params: Optional[dict] = None, bit_depth: int = 8,
               force_zero_mv: bool = False) -> dict:
    I = np.ascontiguousarray(I, dtype=np.uint16)
    J = np.ascontiguousarray(J, dtype=np.uint16)
    h, w = I.shape
    B = (w // 8) * (h // 8)
    mv = np.zeros((max(B, 1), 2), np.int8)
    sad = np.zeros(max(B, 1), np.int32)
    ints = np.zeros(9, np.int64)
    dbl = np.zeros(4, np.float64)
    p = make_params(params)
    _check(lib().vsa_debug_pair(C.byref(p), _ptr(I), _ptr(J), w, h, bit_depth, int(force_zero_mv), _ptr(mv),
                                _ptr(sad), _ptr(ints), _ptr(dbl)), "debug_pair")
    keys = ("sx", "sy", "sxx", "syy", "sxy", "n", "a", "B", "static")
    out = {k: int(v) for k, v in zip(keys, ints)}
    out.update(ncc=float(dbl[0]), swr=float(dbl[1]), amm=float(dbl[2]), act=float(dbl[3]))
    out["mv"] = mv[:B].reshape(h // 8, w // 8, 2)
    out["sad"] = sad[:B].reshape(h // 8, w // 8)
    return out


def params_from_json(text: str) -> dict:
    """The library's reading of a JSON parameter object (vsa_params_from_json)."""
    p = Params()
    _check(lib().vsa_params_from_json(text.encode(), C.byref(p)), "params_from_json")
    return {name: getattr(p, name) for name, _ in Params._fields_}


def debug_flow_pair(I: np.ndarray, J: np.ndarray, params: Optional[dict] = None, bit_depth: int = 8) -> dict:
    """Dense inverse search flow pair measure of two host planes (see
    vsa_debug_flow_pair): {"flow": [h, w, 2], "ncc", "swr", "amm", "act", "static"}."""
    I = np.ascontiguousarray(I, dtype=np.uint16)
    J = np.ascontiguousarray(J, dtype=np.uint16)
    h, w = I.shape
    flow = np.zeros((h, w, 2), np.float64)
    dbl = np.zeros(4, np.float64)
    st = C.c_int32(0)
    p = make_params(params)
    _check(lib().vsa_debug_flow_pair(C.byref(p), _ptr(I), _ptr(J), w, h, bit_depth, _ptr(flow), _ptr(dbl),
                                     C.byref(st)), "debug_flow_pair")
    return {"flow": flow, "ncc": float(dbl[0]), "swr": float(dbl[1]), "amm": float(dbl[2]), "act": float(dbl[3]),
            "static": int(st.value)}


def flow_scratch_bytes(w: int, h: int) -> int:
    return _check(lib().vsa_flow_scratch_bytes(w, h), "flow_scratch_bytes")


def flow_pair(I, J, scratch, results, params: Optional[dict] = None, flow=None, stream: Optional[int] = None):
    """Enqueue the flow pair measure of two CUDA tensors [h, w] (uint8, or
    int16/uint16 holding 10-bit samples) into `results` (CUDA float64 [5]),
    using `scratch` (CUDA uint8, at least flow_scratch_bytes) and, if given,
    `flow` (CUDA float64 [h, w, 2])."""
    h, w = I.shape
    bits = 8 if I.element_size() == 1 else 10
    p = make_params(params)
    _check(lib().vsa_flow_pair(C.byref(p), C.c_void_p(I.data_ptr()), C.c_void_p(J.data_ptr()), w, h,
                               I.stride(0) * I.element_size(), bits, C.c_void_p(scratch.data_ptr()),
                               scratch.numel(), None if flow is None else C.c_void_p(flow.data_ptr()),
                               C.c_void_p(results.data_ptr()), None if stream is None else C.c_void_p(stream)),
           "flow_pair")


def debug_finish(ints: np.ndarray, a0: float) -> np.ndarray:
    v = np.ascontiguousarray(ints, dtype=np.int64).reshape(-1, 8)
    out = np.zeros((v.shape[0], 4), np.float64)
    _check(lib().vsa_debug_finish(_ptr(v), v.shape[0], float(a0), _ptr(out)), "debug_finish")
    return out


def debug_decide(seq: dict, params: Optional[dict] = None, dense: bool = False, k_max: int = 0) -> dict:
    p = make_params(params)
    km = k_max or p.k_max
    T = len(seq["act"])
    kw = km + 2
    act = np.ascontiguousarray(seq["act"], np.float64)
    swr = np.ascontiguousarray(seq["swr"], np.float64)
    stat = np.ascontiguousarray(seq["static"], np.uint8)
    v = np.ascontiguousarray(seq["v"], np.float64).reshape(T, 3)
    F = np.ascontiguousarray(seq["F"], np.float64).reshape(T, kw)
    S = np.ascontiguousarray(seq["S"], np.float64).reshape(T, kw)
    P = np.ascontiguousarray(seq["P"], np.float64).reshape(T, kw)
    recs = np.zeros(T, FRAME_DTYPE)
    shots = np.zeros(T + 1, SHOT_DTYPE)
    kcap = T * (4 + 2 * kw) + 16
    keys = np.zeros(kcap, KEY_DTYPE)
    ns, nk = C.c_int32(0), C.c_int32(0)
    _check(lib().vsa_debug_decide(C.byref(p), km, int(dense), T, _ptr(act), _ptr(swr), _ptr(stat), _ptr(v),
                                  _ptr(F), _ptr(S), _ptr(P), _ptr(recs), _ptr(shots), shots.size, C.byref(ns),
                                  _ptr(keys), kcap, C.byref(nk)), "debug_decide")
    return {"frames": recs, "shots": shots[:ns.value].copy(), "keys": keys[:nk.value].copy()}
