"""Benchmark: frames/sec and multiple of real time of the measure engine on
2048x1080 8-bit clips (the 2K workload), one MI355X.

One step = one engine time step over B concurrently analysed 2K streams: every
stream ingests one frame (pyramid + fields), its consecutive pair is matched
(motion field, warped moments, NCC/SWR/AMM/ACT), the sparse measures planned
by the previous step (field pairs of analysed frames, deep-check pairs) run,
and the decisions advance.  Input frames are resident in HBM before timing
(a seeded synthetic 1500-frame 2K clip; stream i starts at frame i*1500/B and
wraps around) and are handed to the engine by device pointer.

Printed JSON also carries:
  roofline      the dominant kernel against its roofline (HIP-event times of
                that kernel on the engine stream, algorithmic bytes or
                absolute differences per launch);
  cpu_baseline  the CPU oracle on a bounded sample of the same clip;
  plain_fps     the same clip as one stream (no cross-stream batching).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s; v_sad_u8 folds 4 absolute
# differences into one full-rate lane-op (v_qsad_pk_u16_u8: 16 at quarter rate)
AD_PEAK_T = 256 * 64 * 2.4e9 * 4 / 1e12
RT_FPS = 25.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pyramid_k_me_2k_b256_traffic.txt")
K1_SOURCE = os.path.join(ROOT, "paper_2502_09202_amd", "csrc", "k_pyramid.hip")
ME_SOURCE = os.path.join(ROOT, "paper_2502_09202_amd", "csrc", "k_me.hip")


def me_traffic(streams):
    """HBM bytes per motion-search launch (mean of the consecutive and the
    sparse launch) from the same counter summary, or None if k_me.hip has
    changed since the counters were taken or they were taken at another
    batch size."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(ME_SOURCE, "rb").read()).hexdigest()
        if kv.get("k_me.hip sha256") != sha or int(kv.get("streams", -1)) != streams:
            return None
        return float(kv["k_me hbm bytes per launch"])
    except (OSError, KeyError, ValueError):
        return None


def k1_traffic(streams):
    """HBM bytes per pyramid launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by the copy-kernel factor),
    or None if the kernel source has changed since the counters were taken or
    they were taken at another batch size."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(K1_SOURCE, "rb").read()).hexdigest()
        if kv.get("k_pyramid.hip sha256") != sha or int(kv.get("streams", -1)) != streams:
            return None
        return float(kv["hbm bytes per launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_only(nbytes, reps):
    """A plain device copy of known size: the calibration run for the HBM byte
    counters (FETCH_SIZE / WRITE_SIZE of one dispatch vs nbytes)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}))


def _spec(kind):
    import synth
    _, seed, T, W, H = kind                   # the 2K clip
    return synth.make_c2(seed=seed, T=T, W=W, H=H, k_dis=8)


def _render_range(args):
    kind, n, lo, hi, shm_name = args
    from multiprocessing import shared_memory
    import synth
    spec = _spec(kind)
    r = synth.Renderer(spec)
    shm = shared_memory.SharedMemory(name=shm_name)
    out = np.ndarray((n, spec.H, spec.W), np.uint8 if spec.bits == 8 else np.uint16, buffer=shm.buf)
    for t in range(lo, hi):
        out[t] = r.frame(t)
    del out
    shm.close()
    return hi - lo


def render_frames(kind, n, W, H, workers, bits=8):
    """Frames 0..n-1 of a seeded clip, rendered in parallel processes."""
    from multiprocessing import shared_memory
    dt = np.uint8 if bits == 8 else np.uint16
    shm = shared_memory.SharedMemory(create=True, size=n * H * W * np.dtype(dt).itemsize)
    try:
        chunks = np.linspace(0, n, workers * 4 + 1).astype(int)
        jobs = [(kind, n, int(a), int(b), shm.name) for a, b in zip(chunks[:-1], chunks[1:]) if b > a]
        with mp.get_context("spawn").Pool(workers) as pool:
            done = sum(pool.map(_render_range, jobs))
            pool.close()          # workers exit on their own; the with-exit then terminates nothing
            pool.join()
        assert done == n
        frames = np.ndarray((n, H, W), dt, buffer=shm.buf).copy()
    finally:
        shm.close()
        shm.unlink()
    return frames


def render_clip(seed, T, W, H, workers):
    return render_frames(("c2", seed, T, W, H), T, W, H, workers)


def mix_clips(n, frames_needed, torch, seed=3, first=0):
    """Clips first..first+n-1 of the uneven mix, each rendered on the device
    from its own spec (format i mod 6, length U{200..3000}): its first
    min(length, frames_needed) frames, or all of them (frames_needed None)."""
    import synth
    from synth.device import DeviceRenderer
    clips = []
    for i in range(first, first + n):
        spec = synth.make_mix_clip(i, seed=seed)
        m = spec.T if frames_needed is None else min(spec.T, frames_needed)
        clips.append(DeviceRenderer(spec, "cuda:0").frames(0, m))
    torch.cuda.synchronize()
    return clips


def run_mix(vsa, clips, params, steps, warmup, torch):
    """The clips of the uneven mix in one engine, one stream each, every
    stream stepping together from its clip's first frame; a clip shorter than
    the run ends there (its stream is ended after its last frame and pushes no
    more).  Returns frames/s (frames pushed in the timed steps) and the
    per-kernel times."""
    B = len(clips)
    e = vsa.Engine(device=0, max_streams=B, params=params, profile=2)
    sids, bases, pitches, planes, nsrc = [], [], [], [], []
    for src in clips:
        F, H, W = src.shape
        sids.append(e.stream_open(W, H, 8))
        bases.append(src.data_ptr()); pitches.append(W); planes.append(H * W); nsrc.append(F)
    sids = np.array(sids, np.int32)
    bases = np.array(bases, np.uint64); pitches = np.array(pitches, np.int64)
    planes = np.array(planes, np.uint64); nsrc = np.array(nsrc, np.int64)

    def do_step(s):
        live = s < nsrc
        if not live.any():
            e.step()
            return 0
        ptrs = bases[live] + np.uint64(s) * planes[live]
        if e.stream_push_batch(sids[live], ptrs, pitches[live], vsa.SRC_DEVICE_BORROW, None) != 0:
            raise RuntimeError(vsa.last_error())
        for sid in sids[s == nsrc - 1]:
            e.stream_end(int(sid))
        e.step()
        return int(live.sum())

    for s in range(warmup):
        do_step(s)
    e.sync()
    e.kernel_times(reset=True)
    pushed = 0
    t0 = time.perf_counter()
    for s in range(warmup, warmup + steps):
        pushed += do_step(s)
    e.sync()
    dt = time.perf_counter() - t0
    kt = e.kernel_times()
    e.close()
    return pushed / dt, pushed, {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items() if v[1]}


def flow_ops(w, h):
    """Double-precision operations of one dense-flow pair measure of a w x h
    pair (the kernels' arithmetic, counted per operation: add, sub, mul, div,
    sqrt, min, max, floor, abs): a bilinear sample is 17; an inverse-
    compositional step is 26 per patch pixel plus 16 for the 2 x 2 solve; a
    patch's Hessian 8 per pixel; densification 28 per covering patch of a
    pixel plus 2; the measure sums 32 per pixel.  Scales: the pair's and up to
    two box-downscaled copies at least 8 x 8."""
    def origins(n):
        if n < 8:
            return 0
        k = (n - 8) // 4 + 1
        return k + (1 if (k - 1) * 4 + 8 < n else 0)

    def cover(n):
        k = (n - 8) // 4 + 1
        extra = origins(n) > k
        tot = 0
        for x in range(n):
            lo = (x - 4) // 4 if x >= 8 else 0
            hi = min(k - 1, x // 4)
            tot += max(0, hi - lo + 1) + (1 if extra and x >= n - 8 else 0)
        return tot

    ops = 0
    cw, ch = w, h
    for k in range(3):
        if k > 0:
            cw, ch = cw // 2, ch // 2
            if cw < 8 or ch < 8:
                break
        npatch = origins(cw) * origins(ch)
        ops += npatch * (64 * 8 + 8 * (64 * 26 + 16) + 2)
        ops += cover(cw) * cover(ch) * 28 + 2 * cw * ch
    return ops + 32 * w * h


def run_flow(vsa, dev_frames, params, torch, pairs=64, warmup=8):
    """Dense-flow pair measures (search = 2) of consecutive 2K frames at the
    working level (512 x 270, two box steps of the frames, formed on the device
    before timing), one after another on one HIP stream; returns pairs/s, ms
    per pair and the double-precision operation rate."""
    x = dev_frames[: pairs + warmup + 1].to(torch.int32)
    for _ in range(2):
        x = (x[:, 0::2, 0::2][:, : x.shape[1] // 2, : x.shape[2] // 2] + x[:, 1::2, 0::2][:, : x.shape[1] // 2, : x.shape[2] // 2]
             + x[:, 0::2, 1::2][:, : x.shape[1] // 2, : x.shape[2] // 2] + x[:, 1::2, 1::2][:, : x.shape[1] // 2, : x.shape[2] // 2]
             + 2) >> 2
    lv = x.to(torch.uint8).contiguous()
    n, h, w = lv.shape
    p = dict(params, search=2)
    scratch = torch.empty(vsa.flow_scratch_bytes(w, h), dtype=torch.uint8, device="cuda:0")
    res = torch.zeros((n, 5), dtype=torch.float64, device="cuda:0")
    st = torch.cuda.Stream()
    for t in range(warmup):
        vsa.flow_pair(lv[t], lv[t + 1], scratch, res[t], p, stream=st.cuda_stream)
    st.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for t in range(warmup, warmup + pairs):
        vsa.flow_pair(lv[t], lv[t + 1], scratch, res[t], p, stream=st.cuda_stream)
    e1.record(st)
    st.synchronize()
    ms = e0.elapsed_time(e1) / pairs
    ops = flow_ops(w, h)
    return {"workload": f"dense inverse search flow pair measure (search = 2) of consecutive frames of the 2K clip "
                        f"at the working level ({w} x {h}, 8-bit), one pair after another on one HIP stream",
            "pairs_per_s": round(1e3 / ms, 1), "ms_per_pair": round(ms, 4),
            "fp64_ops_per_pair": ops, "fp64_gops": round(ops / (ms * 1e-3) / 1e9, 2),
            "fp64_peak_gops": 78600.0, "frac": round(ops / (ms * 1e-3) / 1e9 / 78600.0, 5)}


def run_stress(vsa, params, B, frames_per_stream, seg, torch,
               configs=(("sparse", False, 0), ("dense", True, 0))):
    """The 4K 10-bit 50i clip (its full length) cut into B consecutive pieces,
    piece s read by stream s in order, in two engines at once (sparse and dense
    schedule).  Each segment of `seg` steps is rendered on the device first,
    untimed; each engine's steps over it are timed between device
    synchronisations.  Returns, per schedule, frames/s, AD per frame and the
    per-kernel times, and the render time.  Each config is (name, dense,
    search); per config the result is frames/s, 8 x 8 blocks searched per
    frame and the per-kernel times."""
    import synth
    from synth.device import DeviceRenderer
    T = B * frames_per_stream
    spec = synth.make_c5(seed=5, T=T)
    H, W = spec.H, spec.W
    rends = [DeviceRenderer(spec, "cuda:0") for _ in range(B)]
    buf = torch.empty((B, seg, H, W), dtype=torch.int16, device="cuda:0")
    engines = {}
    for name, dense, search in configs:
        e = vsa.Engine(device=0, max_streams=B, params=dict(params, search=search), profile=2,
                       schedule=vsa.SCHEDULE_DENSE if dense else vsa.SCHEDULE_SPARSE)
        engines[name] = (e, np.array([e.stream_open(W, H, 10) for _ in range(B)], np.int32))
    pitches = np.full(B, W * 2, np.int64)
    plane = H * W * 2
    base = np.array([buf[b].data_ptr() for b in range(B)], np.uint64)
    c0 = {d: e.counters() for d, (e, _) in engines.items()}
    for e, _ in engines.values():
        e.kernel_times(reset=True)
    busy = {name: 0.0 for name in engines}
    render_s = 0.0
    done = 0
    while done < frames_per_stream:
        n = min(seg, frames_per_stream - done)
        t1 = time.perf_counter()
        for b in range(B):
            rends[b].render_into(buf[b, :n], b * frames_per_stream + done)
        torch.cuda.synchronize()
        render_s += time.perf_counter() - t1
        for name, (e, sids) in engines.items():
            e.sync()
            t1 = time.perf_counter()
            for j in range(n):
                if e.stream_push_batch(sids, base + np.uint64(j * plane), pitches, vsa.SRC_DEVICE_BORROW,
                                       None) != 0:
                    raise RuntimeError(vsa.last_error())
                if done + j == frames_per_stream - 1:
                    for sid in sids:
                        e.stream_end(int(sid))
                e.step()
            e.sync()
            busy[name] += time.perf_counter() - t1
        done += n
    out = {}
    for name, (e, sids) in engines.items():
        c1 = e.counters()
        kt = e.kernel_times()
        blocks = (c1["consecutive_blocks"] - c0[name]["consecutive_blocks"]) + \
                 (c1["sparse_blocks"] - c0[name]["sparse_blocks"])
        out[name] = (B * frames_per_stream / busy[name], blocks / (B * frames_per_stream),
                     {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items() if v[1]})
        e.close()
    return out, render_s


def serve_requests(serve, clips, rate, seed):
    """One request per rendered clip, arriving as a Poisson process at `rate`
    per second (all at once for rate 0), each reading its own clip from its
    first frame to its last."""
    arr = serve.poisson_arrivals(rate, len(clips), seed) if rate > 0 else np.zeros(len(clips))
    return [serve.ClipRequest(cid, float(arr[cid]), src, 0, int(src.shape[0]), 8)
            for cid, src in enumerate(clips)]


def geometry(W, H, params):
    """Pyramid geometry of a W x H stream (the engine's level rule): level
    sizes halve with the odd row / column dropped; the working level L is the
    first no wider than wmax, the field level Lf = max(0, L - lf_offset), and
    Lcap the coarsest level still holding 2 x 2 blocks of 8 x 8."""
    dims = [(W, H)]
    while dims[-1][0] > 1 and dims[-1][1] > 1:
        dims.append((dims[-1][0] // 2, dims[-1][1] // 2))
    L = next(i for i, (w, _) in enumerate(dims) if w <= params["wmax"])
    Lcap = max(i for i, (w, h) in enumerate(dims) if i >= L and w // 8 >= 2 and h // 8 >= 2)
    Lf = max(0, L - params["lf_offset"])
    return {"L": L, "Lcap": Lcap, "Lf": Lf, "dims": dims, "field": (W >> Lf, (H // 2) >> Lf)}


def k1_tiles(g):
    """Pyramid tiles of one frame (64 x 16 working-level pixels up to L = 2,
    32 x 16 at L = 3, 16 x 16 beyond; the grid also covers the fields)."""
    L, Lf = g["L"], g["Lf"]
    wl, hl = g["dims"][L]
    wf, _ = g["field"]
    shift = L - Lf
    gw = max((wf + (1 << shift) - 1) >> shift, wl)
    tw = 16 * (4 if L <= 2 else (2 if L == 3 else 1))
    return -(-gw // tw) * -(-hl // 16)


def k1_bytes_per_frame(g, W, H, k_max, intensity=True):
    """Algorithmic bytes of the pyramid kernel for one 8-bit frame: the luma
    plane read once, the stored levels L..L+ceil(log2(k_max+1)) and both fields
    written, and (with the intensity measure) one 256-bin uint16 histogram
    written per tile."""
    L, Lcap = g["L"], g["Lcap"]
    ltop = min(L + int(np.ceil(np.log2(k_max + 1))), Lcap)
    b = W * H
    for l in range(L, ltop + 1):
        w, h = g["dims"][l]
        b += w * h
    wf, hf = g["field"]
    return b + 2 * wf * hf + (k1_tiles(g) * 256 * 2 if intensity else 0)


# Untimed steps before any timed window.  Every stream opens a shot at its
# first frame, so for the first n_ss + k_max + a few steps all streams analyse
# their first shot's fields at once (about 4x the sparse work of the steady
# state), and the engine's launch tuner times its candidates from step 64 to
# about step 160; the timed steps start after both, whatever --warmup says.
PREROLL_STEPS = 200
MARKER = "spin_kernel"     # torch.cuda._sleep's kernel: brackets the timed steps in a kernel trace
# The headline times the pyramid and motion-search launches of one step in
# this many (timing events stamped by a dispatch cost it device time; every
# step timed costs the headline several percent).
PROFILE_EVERY = 1


def mark(torch):
    """A tiny, uniquely named kernel on the device (torch.cuda._sleep), with
    the device idle before and after it: the boundaries of the headline's
    timed steps in a rocprofv3 trace or counter run of this command."""
    torch.cuda.synchronize()
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()


def run_engine(vsa, dev_frames, params, B, steps, warmup, profile, torch, preroll=PREROLL_STEPS, markers=False,
               src=None, **engine_kw):
    """B streams of the resident clip (stream i starts at frame i*F/B), `preroll
    + warmup` untimed steps, then `steps` timed ones.  src: None reads the
    frames in place from device memory; a pinned host tensor of the same clip
    makes every step upload its planes from host memory (end-to-end rate)."""
    F, H, W = dev_frames.shape
    e = vsa.Engine(device=0, max_streams=max(B, 1), params=params, profile=int(profile), **engine_kw)
    sids = np.array([e.stream_open(W, H, 8) for _ in range(B)], np.int32)
    host = src is not None
    base = (src if host else dev_frames).data_ptr()
    mode = vsa.SRC_HOST_BORROW if host else vsa.SRC_DEVICE_BORROW
    fbytes = H * W
    offs = (np.arange(B) * (F // B)) % F
    pitches = np.full(B, W, np.int64)

    def do_step(s):
        idx = (offs + s) % F
        ptrs = (base + idx.astype(np.uint64) * fbytes).astype(np.uint64)
        rc = e.stream_push_batch(sids, ptrs, pitches, mode, None)
        if rc != 0:
            raise RuntimeError(vsa.last_error())
        e.step()

    for s in range(preroll + warmup):
        do_step(s)
    e.sync()
    torch.cuda.synchronize()
    if profile:
        e.kernel_times(reset=True)
    c0 = e.counters()
    if markers:
        mark(torch)
    t0 = time.perf_counter()
    for s in range(preroll + warmup, preroll + warmup + steps):
        do_step(s)
    e.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if markers:
        mark(torch)
    c1 = e.counters()
    kt = e.kernel_times() if profile else None
    frames_out = sum(len(e.poll_frames(int(sid), 1 << 20)) for sid in sids)
    c1["tuning"] = {b: (v["best"], v["candidates"][v["best"]]["wgs"] if v["best"] >= 0 else None)
                    for b, v in e.tuning().items()} if not engine_kw.get("me_wgs_per_cu") else "fixed"
    e.close()
    return dt, kt, c0, c1, frames_out


def run_clip_leg(vsa, dev_frames, params, chunk, runs, torch):
    """The whole resident clip analysed alone by the offline form, `runs`
    times after one untimed run; frames/s of each run."""
    F, H, W = dev_frames.shape
    out = []
    with vsa.Clip(W, H, chunk=chunk, params=params) as c:
        c.run_tensor(dev_frames)
        c0 = c.counters()
        for _ in range(runs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = c.run_tensor(dev_frames)
            out.append(F / (time.perf_counter() - t0))
        c1 = c.counters()
    per_run = {k: (c1[k] - c0[k]) / runs for k in c0}
    return out, per_run, len(res["shots"])


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_sample(args):
    frames, params = args
    import oracle
    t0 = time.perf_counter()
    oracle.run_clip(frames, params)
    return time.perf_counter() - t0


def cpu_baseline(frames, params, budget_s, copies_max=8):
    """The oracle as it stands (plain scalar C++, one thread per clip) on the
    first frames of the same 2K clip: one process, then min(nproc, 8)
    processes each analysing that sample at once (independent clips are the
    only parallelism the oracle has).  value = the parallel aggregate."""
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    n = 4
    t0 = time.perf_counter()
    oracle.run_clip(frames[:n], params)
    per = (time.perf_counter() - t0) / n
    n = int(max(8, min(len(frames), budget_s / max(per, 1e-6))))
    sample = np.ascontiguousarray(frames[:n])
    dt1 = _oracle_sample((sample, params))
    nproc = os.cpu_count() or 1
    copies = max(1, min(nproc, copies_max))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(copies) as pool:
        times = pool.map(_oracle_sample, [(sample, params)] * copies)
        pool.close()
        pool.join()
    wall = time.perf_counter() - t0
    agg = copies * n / max(times)
    return {"value": round(agg, 3), "unit": "frames/s", "cores": copies, "kind": "oracle",
            "sample": f"first {n} frames of the 2048x1080 clip (k_max 8, sparse schedule), analysed by "
                      f"{copies} oracle processes at once (one thread each); value = {copies} x {n} frames / "
                      f"slowest process",
            "single_process_fps": round(n / dt1, 3), "per_core_fps": round(agg / copies, 3),
            "x_realtime_single": round(n / dt1 / RT_FPS, 3), "wall_s_parallel": round(wall, 2),
            "nproc": nproc, "cpu_model": _cpu_model()}


def short_kernel_name(name):
    """A kernel's name without the return type, namespaces and parameter list
    (template arguments kept)."""
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("vsa::(anonymous namespace)::", "").replace("vsa::", "")
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def summarize_trace(path, match=None):
    """Per-kernel statistics of a rocprofv3 CSV (kernel trace or counter
    collection) restricted to the dispatches between the two marker kernels
    that bracket the headline's timed steps (dispatch ids strictly between);
    with match, every dispatch of the kernels whose name contains it."""
    import csv
    rows = list(csv.DictReader(open(path)))
    if not rows:
        raise SystemExit(f"{path}: no rows")
    key = "Dispatch_Id" if "Dispatch_Id" in rows[0] else "Correlation_Id"
    if match:
        rows = [r for r in rows if match in r["Kernel_Name"]]
        lo, hi = -1, 1 << 62
    else:
        marks = sorted({int(r[key]) for r in rows if MARKER in r["Kernel_Name"]})
        if len(marks) < 2:
            raise SystemExit(f"{path}: {len(marks)} marker dispatches (need 2)")
        lo, hi = marks[0], marks[1]
    win = [r for r in rows if lo < int(r[key]) < hi]
    out = {}
    if "Counter_Name" in rows[0]:
        for r in win:
            d = out.setdefault((r["Kernel_Name"], r["Counter_Name"]), {})
            d[int(r[key])] = d.get(int(r[key]), 0.0) + float(r["Counter_Value"])
        print(f"# {path}: " + (f"every dispatch of kernels matching {match!r}" if match else
                                   f"dispatches {lo + 1}..{hi - 1} (between the markers)"))
        print(f"# {'kernel':<44} {'counter':<12} {'dispatches':>10} {'mean per dispatch':>18}")
        for (k, c), d in sorted(out.items()):
            print(f"  {k[:44]:<44} {c:<12} {len(d):>10} {sum(d.values()) / len(d):>18.1f}")
        return
    for r in win:
        d = out.setdefault(short_kernel_name(r["Kernel_Name"]), [])
        d.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print(f"# {path}: " + (f"every dispatch of kernels matching {match!r}" if match else
                               f"dispatches {lo + 1}..{hi - 1} (between the markers)"))
    print(f"# {'kernel':<44} {'calls':>6} {'total ms':>9} {'avg us':>9} {'min us':>9} {'max us':>9}")
    for k, d in sorted(out.items(), key=lambda kv: -sum(kv[1])):
        print(f"  {k[:44]:<44} {len(d):>6} {sum(d) / 1e3:>9.3f} {sum(d) / len(d):>9.2f} {min(d):>9.2f} {max(d):>9.2f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--streams", type=int, default=256)
    ap.add_argument("--also-streams", type=int, default=64, help="a second batched run at this stream count (0: none)")
    ap.add_argument("--frames", type=int, default=1500)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=300)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--gpu-warm-steps", type=int, default=500,
                    help="untimed steps of a separate engine before the timed run (clocks, code objects)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-stream comparison run")
    ap.add_argument("--no-diag", action="store_true", help="skip the all-kernel timing run")
    ap.add_argument("--no-intensity-leg", action="store_true",
                    help="skip the batched run without the unary intensity measure")
    ap.add_argument("--no-mix", action="store_true", help="skip the uneven-mix batched run")
    ap.add_argument("--no-serve", action="store_true", help="skip the served runs")
    ap.add_argument("--serve-clips", type=int, default=32)
    ap.add_argument("--no-stress", action="store_true", help="skip the 4K 10-bit sparse/dense runs")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-rates", default="0.5,1,2,5,10,20",
                    help="comma-separated Poisson rates of the served sweep ('' for none)")
    ap.add_argument("--stress-frames", type=int, default=45000,
                    help="frames of the 4K 10-bit stress clip (the clip's stated length by default)")
    ap.add_argument("--copy-only", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--no-clip", action="store_true", help="skip the offline single-clip run")
    ap.add_argument("--clip-chunk", type=int, default=256, help="frames per chunk of the offline single-clip run")
    ap.add_argument("--clip-runs", type=int, default=5)
    ap.add_argument("--clip-only", action="store_true",
                    help="only the offline single-clip run (one JSON line of its own; for kernel traces)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--preroll", type=int, default=PREROLL_STEPS,
                    help="untimed steps before the warm-up steps of every batched run (first-shot transient)")
    ap.add_argument("--me-wgs", type=int, default=0,
                    help="persistent motion-search workgroups per CU for every batched run (0: the engine's tuner)")
    ap.add_argument("--no-e2e", action="store_true", help="skip the end-to-end run from pinned host memory")
    ap.add_argument("--no-hier", action="store_true", help="skip the coarse-to-fine (search = 1) batched run")
    ap.add_argument("--no-flow", action="store_true", help="skip the dense-flow pair measure timing")
    ap.add_argument("--no-flow-engine", action="store_true",
                    help="skip the batched run with the dense flow for every pair (search = 2)")
    ap.add_argument("--flow-steps", type=int, default=20, help="timed steps of the dense-flow batched run")
    ap.add_argument("--flow-engine-only", action="store_true",
                    help="only the dense-flow batched run (one JSON line with it)")
    ap.add_argument("--e2e-steps", type=int, default=40)
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="print per-kernel figures of a rocprofv3 kernel-trace or counter CSV of this command "
                         "over the headline's timed steps (between the marker kernels) and exit")
    ap.add_argument("--trace-match", metavar="NAME",
                    help="with --summarize-trace: every dispatch of the kernels whose name contains NAME instead")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.trace_match)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); streams shard across "
              "GPUs with no exchange, so run one process per GPU", file=sys.stderr)
        sys.exit(2)

    if args.copy_only:
        copy_only(args.copy_only, 5)
        return

    import torch
    from paper_2502_09202_amd import vsa

    W, H = 2048, 1080
    params = vsa.load_params()
    params["k_max"] = 8   # the 2K workload has 8-frame dissolves
    t0 = time.perf_counter()
    frames = render_clip(args.seed, args.frames, W, H, args.workers)
    print(f"[bench] rendered {frames.shape} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.from_numpy(frames).to("cuda:0")
    torch.cuda.synchronize()

    def clip_leg():
        cf, per, nshots = run_clip_leg(vsa, dev, params, args.clip_chunk, args.clip_runs, torch)
        med = float(np.median(cf))
        print(f"[bench] single clip, chunks of {args.clip_chunk}: {med:.0f} frames/s "
              f"(runs {[round(x) for x in cf]})", file=sys.stderr, flush=True)
        return {"workload": f"one {args.frames}-frame 2048x1080 8-bit clip resident in HBM analysed alone by "
                            f"the offline form (vsa_clip_run), chunks of {args.clip_chunk} frames, k_max 8, "
                            "sparse schedule; median of the runs",
                "fps": round(med, 1), "x_realtime": round(med / RT_FPS, 1), "runs_fps": [round(x, 1) for x in cf],
                "ms_per_clip": round(1e3 * args.frames / med, 3), "chunk": args.clip_chunk, "shots": nshots,
                "per_clip": per}

    def flow_engine_leg():
        # the dense flow for every pair the pass measures, on the headline's streams
        fsteps = max(1, args.flow_steps)
        fdt, _, fc0, fc1, _ = run_engine(vsa, dev, dict(params, search=2), args.streams, fsteps, 4, 0, torch,
                                         preroll=16, markers=args.flow_engine_only)
        gf = geometry(W, H, params)
        wl, hl = gf["dims"][gf["L"]]
        ops = args.streams * flow_ops(wl, hl) * fsteps
        sparse = fc1["sparse_tasks"] - fc0["sparse_tasks"]
        print(f"[bench] dense flow B={args.streams}: {args.streams * fsteps / fdt:.0f} frames/s, "
              f"{1e3 * fdt / fsteps:.2f} ms/step", file=sys.stderr, flush=True)
        return {"workload": f"the headline's {args.streams} streams with search = 2: every pair the pass measures "
                            f"(consecutive {wl} x {hl} pairs, field and deep-check pairs) takes the dense inverse "
                            "search flow measure, as pair lists cut into plane rows, one launch per phase and list",
                "fps": round(args.streams * fsteps / fdt, 1), "ms_per_step": round(1e3 * fdt / fsteps, 4),
                "steps": fsteps, "sparse_pairs_per_step": round(sparse / fsteps, 2),
                "fp64_gops_consecutive_only": round(ops / fdt / 1e9, 1),
                "note": "fp64_gops_consecutive_only counts the consecutive pairs' operations alone (a lower "
                        "bound on the step's rate); peak 78600 fp64 GOP/s"}

    if args.flow_engine_only:
        print(json.dumps({"dense_flow_engine": flow_engine_leg()}))
        return

    if args.clip_only:
        if args.gpu_warm_steps > 0:
            run_engine(vsa, dev, params, args.streams, args.gpu_warm_steps, 0, 0, torch)
        print(json.dumps({"single_clip": clip_leg()}))
        return

    if args.gpu_warm_steps > 0:
        # the GPU sat idle while the frames were rendered on the host: a run
        # straight after that is slower by up to a third until the clocks rise
        run_engine(vsa, dev, params, args.streams, args.gpu_warm_steps, 0, 0, torch, preroll=0)
    # the headline: kernel launches timed by events their own dispatch stamps
    # (no extra commands on the streams), the timed steps bracketed by marker
    # kernels for the trace and counter runs of this same command
    dt, kt, c0, c1, nout = run_engine(vsa, dev, params, args.streams, args.steps, args.warmup,
                                      0 if args.no_profile else 1, torch, preroll=args.preroll, markers=True,
                                      profile_every=PROFILE_EVERY, me_wgs_per_cu=args.me_wgs)
    fps = args.streams * args.steps / dt
    print(f"[bench] batched B={args.streams}: {fps:.0f} frames/s, {1e3 * dt / args.steps:.3f} ms/step, "
          f"{nout} records", file=sys.stderr, flush=True)
    extra = {}
    if not args.no_profile:
        # the same run with the engine's timing events off: what the sampled
        # events cost
        odt, _, _, _, _ = run_engine(vsa, dev, params, args.streams, args.steps, args.warmup, 0, torch,
                                     preroll=args.preroll, me_wgs_per_cu=args.me_wgs)
        extra["events_off"] = {"fps": round(args.streams * args.steps / odt, 1),
                               "ms_per_step": round(1e3 * odt / args.steps, 4)}
        print(f"[bench] batched B={args.streams}, timing events off: {args.streams * args.steps / odt:.0f} "
              "frames/s", file=sys.stderr, flush=True)
    if args.also_streams > 0:
        adt, _, _, _, _ = run_engine(vsa, dev, params, args.also_streams, args.steps, args.warmup, 0, torch,
                                     preroll=args.preroll)
        afps = args.also_streams * args.steps / adt
        extra[f"batched_{args.also_streams}_streams"] = {"fps": round(afps, 1),
                                                         "x_realtime_per_stream": round(afps / args.also_streams / RT_FPS, 1),
                                                         "ms_per_step": round(1e3 * adt / args.steps, 4)}
        print(f"[bench] batched B={args.also_streams}: {afps:.0f} frames/s", file=sys.stderr, flush=True)
    if not args.no_hier:
        # the coarse-to-fine motion field (search = 1) on the headline's streams
        hp = dict(params, search=1, refine=1)
        hdt, hkt, _, _, _ = run_engine(vsa, dev, hp, args.streams, args.steps, args.warmup, 1, torch,
                                       preroll=args.preroll)
        gh = geometry(W, H, params)
        wl, hl = gh["dims"][gh["L"]]
        ad_pair = ((wl // 2) // 8) * ((hl // 2) // 8) * 289 * 64 + (wl // 8) * (hl // 8) * 9 * 64
        ad_full = (wl // 8) * (hl // 8) * 289 * 64
        ms, n = hkt["me8"]
        avg = ms / max(n, 1)
        adl = args.streams * ad_pair
        extra["coarse_to_fine"] = {
            "workload": f"the headline's {args.streams} streams with search = 1: frame pairs take the full search "
                        "on the box-downscaled pair, then +-1 around twice that vector (reach 17 working pixels, "
                        "68 px at 2K, against 8 for the full search); field pairs keep the full search",
            "fps": round(args.streams * args.steps / hdt, 1), "ms_per_step": round(1e3 * hdt / args.steps, 4),
            "consecutive_launch": {"kernel": "k_me_hier<uint8_t>", "avg_launch_us": round(avg * 1e3, 3),
                                   "ad_per_launch": adl, "achieved": round(adl / (avg * 1e-3) / 1e12, 2),
                                   "frac": round(adl / (avg * 1e-3) / 1e12 / AD_PEAK_T, 4)},
            "ad_per_pair": ad_pair, "ad_per_pair_full_search": ad_full}
        print(f"[bench] coarse-to-fine B={args.streams}: {args.streams * args.steps / hdt:.0f} frames/s, "
              f"consecutive launch {avg * 1e3:.1f} us", file=sys.stderr, flush=True)
    if not args.no_flow:
        extra["dense_flow_pair"] = run_flow(vsa, dev, params, torch)
        print(f"[bench] dense flow pair: {extra['dense_flow_pair']['ms_per_pair']:.3f} ms per 512x270 pair",
              file=sys.stderr, flush=True)
    if not args.no_flow_engine:
        extra["dense_flow_engine"] = flow_engine_leg()
    if not args.no_intensity_leg:
        # the same batched run without the unary intensity measure (no decision uses it)
        ndt, _, _, _, _ = run_engine(vsa, dev, params, args.streams, args.steps, args.warmup, 0, torch,
                                     preroll=args.preroll, no_intensity=1)
        extra["batched_no_intensity"] = {"fps": round(args.streams * args.steps / ndt, 1),
                                         "ms_per_step": round(1e3 * ndt / args.steps, 4)}
        print(f"[bench] batched B={args.streams} without the intensity measure: "
              f"{args.streams * args.steps / ndt:.0f} frames/s", file=sys.stderr, flush=True)
    if not args.no_e2e and args.e2e_steps > 0:
        # end to end: every step uploads its planes from pinned host memory
        # (VSA_SRC_HOST_BORROW, one DMA per plane, no host-side copy)
        pinned = torch.from_numpy(frames).pin_memory()
        edt, _, _, _, _ = run_engine(vsa, dev, params, args.streams, args.e2e_steps, 5, 0, torch,
                                     preroll=args.preroll // 4, src=pinned)
        efps = args.streams * args.e2e_steps / edt
        extra["end_to_end_pinned_host"] = {
            "workload": f"the headline's {args.streams} streams with every plane uploaded from pinned host "
                        "memory by the step (Y plane only, one host-to-device copy each)",
            "fps": round(efps, 1), "x_realtime": round(efps / RT_FPS, 1),
            "upload_GBps": round(efps * W * H / 1e9, 2), "steps": args.e2e_steps}
        print(f"[bench] end to end from pinned host memory: {efps:.0f} frames/s", file=sys.stderr, flush=True)
        del pinned
    plain_fps = None
    if not args.no_plain and args.plain_steps > 0:
        pdt, _, _, _, _ = run_engine(vsa, dev, params, 1, args.plain_steps, 20, 0, torch, preroll=0)
        plain_fps = args.plain_steps / pdt
        print(f"[bench] plain 1 stream: {plain_fps:.0f} frames/s", file=sys.stderr, flush=True)
    if not args.no_clip:
        extra["single_clip"] = clip_leg()
        if plain_fps:
            extra["single_clip"]["vs_plain_stream"] = round(extra["single_clip"]["fps"] / plain_fps, 2)
    kt_all = None
    if not args.no_diag:
        # untimed diagnostic: every kernel timed, for the per-kernel breakdown
        _, kt_all, _, _, _ = run_engine(vsa, dev, params, args.streams, min(args.steps, 200), 20, 2, torch,
                                        preroll=args.preroll)

    g = geometry(W, H, params)
    k1b = k1_bytes_per_frame(g, W, H, params["k_max"])
    roof = None
    if kt:
        k1_ms, k1_n = kt["pyramid"]
        # k_me runs twice per step (consecutive pairs on one stream, the planned sparse pairs on
        # another); its average launch covers both, as a kernel trace averages them
        me_ms = kt["me8"][0] + kt["me_sparse"][0]
        me_n = kt["me8"][1] + kt["me_sparse"][1]
        step_ms, step_n = kt["step"]
        k1_avg = k1_ms / max(k1_n, 1)
        k1_gbs = args.streams * k1b / (k1_avg * 1e-3) / 1e9
        cblocks = c1["consecutive_blocks"] - c0["consecutive_blocks"]
        sblocks = c1["sparse_blocks"] - c0["sparse_blocks"]
        # absolute differences per launch: every timed step runs one launch of
        # each kind; the durations come from the sampled (timed) steps
        ad = (cblocks + sblocks) * 289 * 64
        ad_launch = ad / (2 * args.steps)
        me_avg_ms = me_ms / max(me_n, 1)
        me_tads = ad_launch / (me_avg_ms * 1e-3) / 1e12 if me_ms > 0 else 0.0
        traffic = k1_traffic(args.streams)
        hbm = {"bound": "hbm", "kernel": "k_pyramid", "achieved": round(k1_gbs, 1), "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": round(k1_gbs / HBM_PEAK_GBS, 4),
               "traffic": None if traffic is None else int(traffic),
               "avg_launch_us": round(k1_avg * 1e3, 3), "bytes_per_launch": args.streams * k1b}
        launches = {}
        for name, key, nb in (("consecutive", "me8", cblocks), ("sparse", "me_sparse", sblocks)):
            ms, n = kt[key]
            avg = ms / max(n, 1)
            adl = nb * 289 * 64 / args.steps
            launches[name] = {"avg_launch_us": round(avg * 1e3, 3), "timed_launches": n, "ad_per_launch": adl,
                              "achieved": round(adl / (avg * 1e-3) / 1e12, 2) if ms > 0 else 0.0}
        alu = {"bound": "alu", "kernel": "k_me<uint8_t>",
               "achieved": round(me_tads, 2), "peak": round(AD_PEAK_T, 1),
               "unit": "T absdiff/s", "frac": round(me_tads / AD_PEAK_T, 4),
               "traffic": None if me_traffic(args.streams) is None else int(me_traffic(args.streams)),
               "avg_launch_us": round(me_avg_ms * 1e3, 3), "ad_per_launch": ad_launch,
               "timed_launches": me_n, "launches": launches}
        roof, other = (hbm, alu) if k1_ms >= me_ms else (alu, hbm)
        extra["roofline_other"] = other
        if kt_all:
            extra["kernel_ms_per_step"] = {k: round(v[0] / max(v[1], 1), 4) for k, v in kt_all.items() if v[1]}
        extra["step_hbm_frac"] = round(args.streams * k1b / (dt / args.steps) / 1e9 / HBM_PEAK_GBS, 4)
    if not args.no_mix:
        t1 = time.perf_counter()
        mix_steps, mix_warm = 300, 30
        clips = mix_clips(64, mix_steps + mix_warm, torch)
        rs = time.perf_counter() - t1
        print(f"[bench] mix: 64 clips rendered in {rs:.1f}s", file=sys.stderr, flush=True)
        mfps, mframes, mkt = run_mix(vsa, clips, dict(params, k_max=8), mix_steps, mix_warm, torch)
        extra["mix"] = {"workload": "clips 0..63 of the uneven mix (720x576i, 1280x720p, 1920x1080p, "
                                    "1920x1080i, 2048x1080p, 3840x2160p; 8-bit; lengths U{200..3000}), each "
                                    "rendered from its own spec, one stream each in one engine, all stepping "
                                    "together from their first frame; a clip that ends stops pushing",
                        "fps": round(mfps, 1), "frames": mframes, "steps": mix_steps,
                        "kernel_ms_per_step": mkt, "render_s": round(rs, 1)}
        del clips
        torch.cuda.empty_cache()
        print(f"[bench] mix 64 clips: {mfps:.0f} frames/s", file=sys.stderr, flush=True)
    if not args.no_serve:
        from paper_2502_09202_amd import serve
        t1 = time.perf_counter()
        clips = mix_clips(args.serve_clips, None, torch, seed=4)
        rs = time.perf_counter() - t1
        nfr = sum(int(c.shape[0]) for c in clips)
        print(f"[bench] serve: {len(clips)} clips ({nfr} frames) rendered in {rs:.1f}s", file=sys.stderr,
              flush=True)
        sv = {}
        p8 = dict(params, k_max=8)

        def serve_once(reqs, path):
            S = serve.Server if path == "batched" else serve.PlainServer
            srv = S(max_streams=256, params=p8)
            try:
                return srv.run(reqs, keep_records=False).summary()
            finally:
                srv.close()

        rates = [float(x) for x in args.serve_rates.split(",") if x] if args.serve_rates else []
        if args.serve_rate not in rates:
            rates.append(args.serve_rate)
        sweep = {}
        for rate in sorted(rates):
            # enough clips for a few seconds of arrivals (all of them at the higher rates)
            n = min(len(clips), max(6, int(round(4 * rate))))
            row = {"clips": n}
            for path in ("batched", "plain"):
                sm = serve_once(serve_requests(serve, clips[:n], rate, 4), path)
                row[path] = sm
                print(f"[bench] serve rate {rate}/s {path}: {sm['fps']:.0f} frames/s, frame p50/p99 "
                      f"{sm['frame_latency_ms_p50']:.2f}/{sm['frame_latency_ms_p99']:.2f} ms", file=sys.stderr,
                      flush=True)
            sweep[f"{rate:g}"] = row
            if rate == args.serve_rate:
                sv["poisson_batched"], sv["poisson_plain"] = row["batched"], row["plain"]
        for path in ("batched", "plain"):
            sv[f"archive_{path}"] = serve_once(serve_requests(serve, clips, 0.0, 4), path)
            print(f"[bench] serve archive {path}: {sv[f'archive_{path}']['fps']:.0f} frames/s", file=sys.stderr,
                  flush=True)
        extra["serve"] = {"workload": f"{len(clips)} clips of the uneven mix at their own lengths "
                                      f"(U{{200..3000}}, {nfr} frames), each rendered from its own spec; "
                                      f"Poisson arrivals at {args.serve_rate}/s (poisson), or all at once "
                                      "(archive); budget 90% of free HBM, 256 slots", "render_s": round(rs, 1),
                          **sv,
                          "rate_sweep": {"note": "per rate, the first max(6, 4 x rate) clips (at most all) "
                                                 "arriving at that Poisson rate, batched and plain per-stream",
                                         **sweep}}
        del clips
        torch.cuda.empty_cache()
    if not args.no_stress:
        B = 8
        per = args.stress_frames // B
        res, rs = run_stress(vsa, dict(params, k_max=4), B, per, 64, torch,
                             configs=(("sparse", False, 0), ("dense", True, 0),
                                      ("sparse_coarse_to_fine", False, 1)))
        st = {"workload": f"the 3840x2160 10-bit (uint16) 50i stress clip, {B * per} frames, cut into {B} "
                          f"consecutive pieces read by {B} streams; low contrast 64..192, pans up to 64 px/frame, "
                          "noise sigma 12, flashes p 1/25, k_max 4; rendered on the device 64 steps at a time, "
                          "untimed", "render_s": round(rs, 1)}
        for name, (sfps, bpf, skt) in res.items():
            row = {"fps": round(sfps, 1), "x_realtime": round(sfps / RT_FPS, 1),
                   "blocks_per_frame": round(bpf, 1), "kernel_ms_per_step": skt}
            if "coarse_to_fine" not in name:            # full search: 289 candidates of 64 samples per block
                row["absdiff_per_frame"] = round(bpf * 289 * 64)
            st[name] = row
            print(f"[bench] 4K 10-bit {name}: {sfps:.0f} frames/s, {bpf:.0f} blocks/frame", file=sys.stderr,
                  flush=True)
        extra["stress_10bit"] = st
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(frames, params, args.cpu_seconds)
        print(f"[bench] cpu oracle: {cpu['value']:.2f} frames/s", file=sys.stderr, flush=True)
    out = {
        "metric": "frames/sec and \u00d7real-time at 2K (1 GPU); p50/p99 frame latency in served mix",
        "value": round(fps, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"2K plain method batched: {args.streams} streams of 2048x1080 8-bit luma, "
                               f"{args.frames}-frame seeded clip resident in HBM, k_max 8, sparse schedule",
                   "streams": args.streams, "width": W, "height": H, "bit_depth": 8},
        "x_realtime": round(fps / RT_FPS, 1),
        "x_realtime_per_stream": round(fps / args.streams / RT_FPS, 1),
        "me_launch": c1.get("tuning"),
        "untimed_steps": {"preroll": args.preroll, "warmup": args.warmup,
                          "why": "every stream opens a shot at its first frame; the preroll takes all of them "
                                 "past that shot's analysis window, so the timed steps are the steady state"},
        "plain_fps": None if plain_fps is None else round(plain_fps, 1),
        "plain_x_realtime": None if plain_fps is None else round(plain_fps / RT_FPS, 1),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if "serve" in extra:
        pb = extra["serve"]["poisson_batched"]
        out["served_frame_latency_ms"] = {"p50": pb["frame_latency_ms_p50"], "p99": pb["frame_latency_ms_p99"],
                                          "mix": "poisson_batched"}
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
