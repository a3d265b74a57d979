"""GPU parity of the unary intensity measure H(t) (Sec. III.A), fused into the
pyramid kernel: per-frame histograms of the working-level image equal the
oracle's bin for bin, and the frame records' mean, standard deviation and mean
absolute deviation equal the oracle's bit for bit.

Cases: one 64 x 16 pyramid tile or less, ragged tiles, every working level the
geometry rule picks for the workload formats (L = 0 .. 3), 8- and 10-bit, a
flat frame (all pixels in one bin), full-range noise (every bin), and several
streams of different shapes in one engine stepping together (each frame's
tiles are summed by that frame's last tile, counted per stream).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _run(vsa, frames_by_stream, params, bits):
    """Push every stream's frames step by step; return the engine and sids."""
    p = dict(params)
    e = vsa.Engine(max_streams=len(frames_by_stream), params=p)
    sids = [e.stream_open(f.shape[2], f.shape[1], bits) for f in frames_by_stream]
    T = max(len(f) for f in frames_by_stream)
    for t in range(T):
        for f, s in zip(frames_by_stream, sids):
            if t < len(f):
                assert e.stream_push(s, f[t], pts=t) == 0
        e.step()
    e.sync()
    return e, sids


def _check_stream(vsa, orc, params, e, sid, frames, bits):
    T = len(frames)
    rs = None
    held = []
    for t in range(T - 1, -1, -1):
        try:
            h = e.histogram(sid, t)
        except vsa.VsaError:
            rs = T - 1 - t
            break
        held.append((t, h))
    assert held, "no frame held"
    g = orc.geometry(frames.shape[2], frames.shape[1], params)
    for t, h in held:
        work = orc.levels(frames[t], params, bits=bits)[("F", g["L"])]
        ref_h, ints, _ = orc.intensity(work, bits)
        assert h.size == 1 << bits
        assert np.array_equal(h.astype(np.int64), ref_h), f"frame {t}"
        assert int(h.sum()) == work.size
    return rs


@pytest.mark.parametrize("W,H,bits,kind", [(64, 32, 8, "noise"), (96, 72, 8, "flat"), (333, 211, 8, "clip"),
                                           (320, 180, 8, "noise"), (1001, 77, 10, "noise"),
                                           (720, 576, 8, "clip"), (640, 360, 10, "clip")])
def test_histograms_and_records(vsa, orc, params, W, H, bits, kind):
    print(f"intensity {W}x{H} {bits}-bit {kind}", flush=True)
    rng = np.random.default_rng(W + H + bits)
    maxv = (1 << bits) - 1
    dt = np.uint8 if bits == 8 else np.uint16
    T = 24
    if kind == "noise":
        frames = rng.integers(0, maxv + 1, size=(T, H, W)).astype(dt)
    elif kind == "flat":
        frames = np.full((T, H, W), rng.integers(0, maxv + 1), dt)
    else:
        spec = synth.make_c5(seed=3, T=T, W=W, H=H) if bits == 10 else synth.make_c2(seed=5, T=T, W=W, H=H)
        frames = synth.render(spec)
    e, (sid,) = _run(vsa, [frames], params, bits)
    _check_stream(vsa, orc, params, e, sid, frames, bits)
    e.stream_end(sid)
    guard = 0
    while not e.stream_done(sid):
        e.step()
        e.sync()
        guard += 1
        assert guard < 100
    got = e.poll_frames(sid, 1000)
    ref = orc.run_clip(frames, params, bits=bits)["frames"]
    assert len(got) == len(ref) == T
    for name in ("h_mean", "h_std", "h_mad"):
        assert np.array_equal(got[name].view(np.uint64), ref[name].view(np.uint64)), name
    e.close()


def test_streams_of_different_shapes_together(vsa, orc, params):
    clips = [synth.render(synth.make_c1(seed=7, T=20)),
             synth.render(synth.make_c2(seed=8, T=20, W=720, H=576)),
             synth.render(synth.make_c2(seed=9, T=20, W=1280, H=720))]
    e, sids = _run(vsa, clips, params, 8)
    for c, s in zip(clips, sids):
        _check_stream(vsa, orc, params, e, s, c, 8)
    e.close()


def test_histogram_argument_checks(vsa, params):
    e = vsa.Engine(max_streams=1, params=params)
    sid = e.stream_open(320, 180, 8)
    with pytest.raises(vsa.VsaError):
        e.histogram(sid, 0)                     # nothing stepped yet
    e.stream_push(sid, np.zeros((180, 320), np.uint8), pts=0)
    e.step()
    e.sync()
    assert e.histogram(sid, 0)[0] == e.histogram(sid, 0).sum()
    with pytest.raises(vsa.VsaError):
        e.histogram(sid, 1)
    with pytest.raises(vsa.VsaError):
        e.histogram(sid + 1, 0)
    e.close()


def test_no_intensity_option(vsa, orc, params):
    """With no_intensity the measure is skipped (NaN, histogram refused) and
    every other output is unchanged."""
    frames = synth.render(synth.make_c1(seed=4, T=16))
    ref = orc.run_clip(frames, params)["frames"]
    e = vsa.Engine(max_streams=1, params=params, no_intensity=1)
    sid = e.stream_open(frames.shape[2], frames.shape[1], 8)
    for t in range(len(frames)):
        assert e.stream_push(sid, frames[t], pts=t) == 0
        if t == len(frames) - 1:
            e.stream_end(sid)
        e.step()
    guard = 0
    while not e.stream_done(sid):
        e.step()
        e.sync()
        guard += 1
        assert guard < 100
    with pytest.raises(vsa.VsaError):
        e.histogram(sid, len(frames) - 1)
    got = e.poll_frames(sid, 100)
    assert len(got) == len(ref)
    for name in ("h_mean", "h_std", "h_mad"):
        assert np.all(np.isnan(got[name])), name
    for name in ("flags", "shot_id", "boundary", "boundary_k", "field_mask", "mom", "n_pix", "amm_num"):
        assert np.array_equal(got[name], ref[name]), name
    for name in ("ncc", "swr", "amm", "act"):
        assert np.array_equal(got[name].view(np.uint64), ref[name].view(np.uint64)), name
    e.close()
