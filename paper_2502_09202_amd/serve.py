"""Served form of the engine: a request loop with continuous batching.

Clips arrive over time (for example as a Poisson process).  An arriving clip
waits in a FIFO queue until the engine admits it: vsa_stream_open succeeds
once a stream slot and enough of the HBM budget are free.  Every engine step
then takes one frame of every admitted clip, so a clip that arrives while
others are on the GPU joins the next step, and a finished clip's slot and
memory are released (without waiting for the device) for the next one.  Each
stream's previous frames, pyramid, fields, measure history and decision state
stay resident in HBM between steps.  Records are published without stalling
the pipeline (vsa_collect) and polled for all streams in one call.

The frames of a clip come from a device tensor (the caller's clip source):
frame k of a request is source[(start + k) % len(source)], read in place.

`PlainServer` is the comparison path: each admitted clip gets its own
single-stream engine (its own HIP streams and its own launches per frame), with
the same admission rule and no cross-stream batching.

Latencies are host clock times: per frame, from the return of the push of that
frame to the record appearing in a poll; per clip, from arrival to its last
record.  Both include the decision lag of the method (a frame's labels are
final only once the frames its checks look ahead to have arrived).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import vsa


@dataclass
class ClipRequest:
    cid: int
    arrival: float            # seconds after the start of the run
    source: object            # CUDA tensor [F, H, W], uint8 (8-bit) or int16/uint16 (10-bit)
    start: int
    length: int
    bit_depth: int = 8
    k_max: int = 0            # 0: the engine's default


@dataclass
class ClipResult:
    cid: int
    arrival: float
    admitted: float
    finished: float
    frames: np.ndarray        # vsa.FRAME_DTYPE records in frame order
    shots: np.ndarray         # vsa.SHOT_DTYPE records


@dataclass
class ServeReport:
    wall_s: float
    frames: int
    fps: float
    steps: int
    frame_latency_ms: np.ndarray
    clip_latency_s: np.ndarray
    queue_wait_s: np.ndarray
    refused_admissions: int
    max_concurrent: int
    results: Dict[int, ClipResult] = field(default_factory=dict)

    def summary(self) -> dict:
        def pct(a, q):
            return float(np.percentile(a, q)) if len(a) else None
        return {
            "clips": len(self.results), "frames": self.frames, "wall_s": round(self.wall_s, 3),
            "fps": round(self.fps, 1), "steps": self.steps, "max_concurrent": self.max_concurrent,
            "frame_latency_ms_p50": pct(self.frame_latency_ms, 50),
            "frame_latency_ms_p99": pct(self.frame_latency_ms, 99),
            "clip_latency_s_p50": pct(self.clip_latency_s, 50),
            "clip_latency_s_p99": pct(self.clip_latency_s, 99),
            "queue_wait_s_p50": pct(self.queue_wait_s, 50),
            "queue_wait_s_p99": pct(self.queue_wait_s, 99),
            "refused_admissions": self.refused_admissions,
        }


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of n clips at Poisson rate `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


class _Clip:
    __slots__ = ("req", "sid", "admit_step", "admitted", "pushed", "ended", "frames", "shots",
                 "plane_bytes", "pitch", "base", "nsrc")

    def __init__(self, req: ClipRequest, sid: int, step: int, now: float):
        self.req = req
        self.sid = sid
        self.admit_step = step
        self.admitted = now
        self.pushed = 0
        self.ended = False
        self.frames: List[np.ndarray] = []
        self.shots: List[np.ndarray] = []
        src = req.source
        self.pitch = src.stride(1) * src.element_size()
        self.plane_bytes = src.stride(0) * src.element_size()
        self.base = src.data_ptr()
        self.nsrc = src.shape[0]

    def next_ptr(self) -> int:
        return self.base + ((self.req.start + self.pushed) % self.nsrc) * self.plane_bytes


def _open(engine: "vsa.Engine", req: ClipRequest) -> Optional[int]:
    H, W = req.source.shape[1], req.source.shape[2]
    try:
        return engine.stream_open(W, H, req.bit_depth, req.k_max)
    except vsa.VsaError as ex:
        if ex.code == vsa.E_ADMIT:
            return None
        raise


class Server:
    """Continuous batching over one engine."""

    def __init__(self, max_streams: int = 256, hbm_budget_bytes: int = 0, params: Optional[dict] = None,
                 device: int = 0):
        self.engine = vsa.Engine(device=device, max_streams=max_streams, hbm_budget_bytes=hbm_budget_bytes,
                                 params=params)

    def close(self):
        self.engine.close()

    def run(self, requests: List[ClipRequest], clock: Callable[[], float] = time.perf_counter,
            keep_records: bool = True, poll_cap: int = 0) -> ServeReport:
        """Serve `requests` to completion.  poll_cap bounds the records taken
        from the engine per step (0: max(4096, 8 x active clips)); whatever a
        finished clip still has queued is drained before its slot is freed."""
        e = self.engine
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque = deque()
        active: Dict[int, _Clip] = {}
        push_time = np.zeros(1024)           # per step: when its pushes returned
        lat: List[np.ndarray] = []
        results: Dict[int, ClipResult] = {}
        qwait: List[float] = []
        refused = 0
        max_conc = 0
        frames_total = 0
        t0 = clock()
        step = 0

        def take(c: _Clip, r: np.ndarray, t_poll: float) -> int:
            lat.append(t_poll - push_time[c.admit_step + r["frame"].astype(np.int64)])
            if keep_records:
                c.frames.append(r)
            return len(r)

        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:                    # FIFO admission
                sid = _open(e, waiting[0])
                if sid is None:
                    refused += 1
                    break
                req = waiting.popleft()
                active[sid] = _Clip(req, sid, step, now)
                qwait.append(now - req.arrival)
            max_conc = max(max_conc, len(active))
            if not active:
                if pending:                   # idle until the next arrival
                    dt = pending[0].arrival - (clock() - t0)
                    if dt > 0:
                        time.sleep(min(dt, 0.01))
                continue
            feed = [c for c in active.values() if c.pushed < c.req.length]
            if feed:
                sids = np.fromiter((c.sid for c in feed), np.int32, len(feed))
                ptrs = np.fromiter((c.next_ptr() for c in feed), np.uint64, len(feed))
                pitches = np.fromiter((c.pitch for c in feed), np.int64, len(feed))
                rc = e.stream_push_batch(sids, ptrs, pitches, vsa.SRC_DEVICE_BORROW, None)
                if rc != 0:
                    raise vsa.VsaError(rc, vsa.last_error())
                for c in feed:
                    c.pushed += 1
            for c in active.values():
                if c.pushed == c.req.length and not c.ended:
                    e.stream_end(c.sid)
                    c.ended = True
            if step == len(push_time):
                push_time = np.concatenate([push_time, np.zeros_like(push_time)])
            push_time[step] = clock() - t0
            e.step()
            step += 1
            e.collect()
            sids, recs = e.poll_frames_all(poll_cap if poll_cap > 0 else max(4096, 8 * len(active)))
            t_poll = clock() - t0
            for sid in np.unique(sids):
                frames_total += take(active[int(sid)], recs[sids == sid], t_poll)
            for sid in [s for s, c in active.items() if c.ended]:
                c = active[sid]
                if e.stream_done(sid):
                    # every record is published; some may still wait in the
                    # stream's queue (the per-step poll is capped): take them
                    # all before the slot (and its queue) is freed
                    while True:
                        r = e.poll_frames(sid, 4096)
                        if not len(r):
                            break
                        frames_total += take(c, r, clock() - t0)
                    shots = e.poll_shots(sid)
                    c.shots.append(shots)
                    done = clock() - t0
                    fr = np.concatenate(c.frames) if c.frames else np.zeros(0, vsa.FRAME_DTYPE)
                    sh = np.concatenate(c.shots) if c.shots else np.zeros(0, vsa.SHOT_DTYPE)
                    results[c.req.cid] = ClipResult(c.req.cid, c.req.arrival, c.admitted, done, fr, sh)
                    e.stream_close(sid)
                    del active[sid]
                elif keep_records:
                    c.shots.append(e.poll_shots(sid))
        wall = clock() - t0
        fl = np.concatenate(lat) * 1e3 if lat else np.zeros(0)
        cl = np.array([r.finished - r.arrival for r in results.values()])
        return ServeReport(wall, frames_total, frames_total / wall if wall > 0 else 0.0, step, fl, cl,
                           np.array(qwait), refused, max_conc, results)


class PlainServer:
    """The per-stream comparison path: one single-stream engine per admitted
    clip (engines are created on demand and reused), the same admission rule
    (a shared HBM budget and a cap on concurrent clips), one launch sequence
    per clip and frame, no cross-stream batching."""

    def __init__(self, max_streams: int = 256, hbm_budget_bytes: int = 0, params: Optional[dict] = None,
                 device: int = 0):
        self.max_streams = max_streams
        self.params = params
        self.device = device
        probe = vsa.Engine(device=device, max_streams=1, params=params)
        self.budget = hbm_budget_bytes or probe.counters()["budget"]
        probe.close()
        self.free: List["vsa.Engine"] = []
        self.used = 0

    def close(self):
        for e in self.free:
            e.close()
        self.free = []

    def run(self, requests: List[ClipRequest], clock: Callable[[], float] = time.perf_counter,
            keep_records: bool = True) -> ServeReport:
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque = deque()
        active: Dict[int, tuple] = {}         # cid -> (engine, sid, clip, footprint, push times)
        lat: List[np.ndarray] = []
        results: Dict[int, ClipResult] = {}
        qwait: List[float] = []
        refused = 0
        max_conc = 0
        frames_total = 0
        rounds = 0
        t0 = clock()
        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:
                req = waiting[0]
                e = self.free.pop() if self.free else vsa.Engine(device=self.device, max_streams=1,
                                                                  params=self.params)
                H, W = req.source.shape[1], req.source.shape[2]
                fp = e.footprint(W, H, req.bit_depth, req.k_max)
                if len(active) >= self.max_streams or self.used + fp > self.budget:
                    self.free.append(e)
                    refused += 1
                    break
                sid = e.stream_open(W, H, req.bit_depth, req.k_max)
                waiting.popleft()
                self.used += fp
                active[req.cid] = (e, sid, _Clip(req, sid, 0, now), fp, [])
                qwait.append(now - req.arrival)
            max_conc = max(max_conc, len(active))
            if not active:
                if pending:
                    dt = pending[0].arrival - (clock() - t0)
                    if dt > 0:
                        time.sleep(min(dt, 0.01))
                continue
            for cid, (e, sid, c, fp, pts) in active.items():
                if c.pushed < c.req.length:
                    rc = e.stream_push_device(sid, c.next_ptr(), c.pitch)
                    if rc != 0:
                        raise vsa.VsaError(rc, vsa.last_error())
                    c.pushed += 1
                    pts.append(clock() - t0)
                    if c.pushed == c.req.length:
                        e.stream_end(sid)
                        c.ended = True
                e.step()
            rounds += 1
            finished = []
            for cid, (e, sid, c, fp, pts) in active.items():
                e.collect()
                sids, recs = e.poll_frames_all()
                if len(recs):
                    t_poll = clock() - t0
                    frames_total += len(recs)
                    lat.append(t_poll - np.asarray(pts)[recs["frame"].astype(np.int64)])
                    if keep_records:
                        c.frames.append(recs)
                if c.ended and e.stream_done(sid):
                    while True:               # drain what the capped poll left
                        r = e.poll_frames(sid, 4096)
                        if not len(r):
                            break
                        frames_total += len(r)
                        lat.append(clock() - t0 - np.asarray(pts)[r["frame"].astype(np.int64)])
                        if keep_records:
                            c.frames.append(r)
                    c.shots.append(e.poll_shots(sid))
                    finished.append(cid)
            for cid in finished:
                e, sid, c, fp, pts = active.pop(cid)
                done = clock() - t0
                fr = np.concatenate(c.frames) if c.frames else np.zeros(0, vsa.FRAME_DTYPE)
                sh = np.concatenate(c.shots) if c.shots else np.zeros(0, vsa.SHOT_DTYPE)
                results[cid] = ClipResult(cid, c.req.arrival, c.admitted, done, fr, sh)
                e.stream_close(sid)
                self.used -= fp
                self.free.append(e)
        wall = clock() - t0
        fl = np.concatenate(lat) * 1e3 if lat else np.zeros(0)
        cl = np.array([r.finished - r.arrival for r in results.values()])
        return ServeReport(wall, frames_total, frames_total / wall if wall > 0 else 0.0, rounds, fl, cl,
                           np.array(qwait), refused, max_conc, results)
