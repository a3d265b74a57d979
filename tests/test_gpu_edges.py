"""Engine edge cases against the oracle (GPU): every stream slot in use at
once, the smallest accepted frame, clips of one to three frames, and a stream
that ends before its first frame.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _drain(e, sids, guard=200):
    for _ in range(guard):
        if all(e.stream_done(int(s)) for s in sids):
            return
        e.step()
        e.sync()
    raise AssertionError("streams did not finish")


def _same(got, ref):
    assert len(got) == len(ref)
    for name in ("frame", "flags", "shot_id", "boundary", "boundary_k", "field_mask", "mom", "n_pix", "amm_num",
                 "n_blocks"):
        assert np.array_equal(got[name], ref[name]), name
    for name in ("ncc", "swr", "amm", "act", "v", "h_mean", "h_std", "h_mad"):
        g, r = got[name], ref[name]
        assert np.array_equal(np.isnan(g), np.isnan(r)), name
        assert np.array_equal(g[~np.isnan(g)].view(np.uint64), r[~np.isnan(r)].view(np.uint64)), name


def _same_shots(got, ref):
    assert len(got) == len(ref)
    for name in ref.dtype.names:
        assert np.array_equal(got[name], ref[name]), name


def _clip(rng, T, H, W, cut=None):
    """Smooth random frames drifting by one pixel per frame, a new scene from `cut` on."""
    base = [rng.integers(0, 256, size=(H + 8, W + 8)), rng.integers(0, 256, size=(H + 8, W + 8))]
    out = np.empty((T, H, W), np.uint8)
    for t in range(T):
        b = base[1 if (cut is not None and t >= cut) else 0]
        out[t] = b[t % 8:t % 8 + H, (2 * t) % 8:(2 * t) % 8 + W]
    return out


def test_every_stream_slot(vsa, orc, params):
    """1024 streams (the slot limit) of 64x32 stepping together; every stream
    ends with one record per frame and sampled streams equal the oracle."""
    M, T, H, W = 1024, 12, 32, 64
    rng = np.random.default_rng(3)
    clips = [_clip(rng, T, H, W, cut=6 if i % 3 == 0 else None) for i in range(M)]
    print("1024 streams", flush=True)
    e = vsa.Engine(max_streams=M, params=params)
    sids = [e.stream_open(W, H, 8) for _ in range(M)]
    for t in range(T):
        for c, s in zip(clips, sids):
            assert e.stream_push(s, c[t], pts=t) == 0
            if t == T - 1:
                e.stream_end(s)
        e.step()
    _drain(e, sids)
    recs = {int(s): e.poll_frames(int(s), 100) for s in sids}
    assert all(len(r) == T for r in recs.values())
    assert all(np.array_equal(r["frame"], np.arange(T)) for r in recs.values())
    for i in (0, 1, 511, 1023):
        ref = orc.run_clip(clips[i], params)
        _same(recs[sids[i]], ref["frames"])
        _same_shots(e.poll_shots(sids[i], 100), ref["shots"])
    e.close()


def test_smallest_frame(vsa, orc, params):
    """16x16 is the smallest frame the geometry accepts (two 8x8 blocks per
    side, 8-row fields); one sample less is refused."""
    rng = np.random.default_rng(5)
    frames = _clip(rng, 10, 16, 16, cut=5)
    e = vsa.Engine(max_streams=2, params=params)
    with pytest.raises(vsa.VsaError):
        e.stream_open(15, 16, 8)
    with pytest.raises(vsa.VsaError):
        e.stream_open(16, 15, 8)
    sid = e.stream_open(16, 16, 8)
    for t in range(len(frames)):
        assert e.stream_push(sid, frames[t], pts=t) == 0
        if t == len(frames) - 1:
            e.stream_end(sid)
        e.step()
    _drain(e, [sid])
    ref = orc.run_clip(frames, params)
    _same(e.poll_frames(sid, 100), ref["frames"])
    _same_shots(e.poll_shots(sid, 100), ref["shots"])
    e.close()


@pytest.mark.parametrize("T", [1, 2, 3])
def test_short_clips(vsa, orc, params, T):
    frames = synth.render(synth.make_c1(seed=8, T=max(T, 2)), range(T))
    ref = orc.run_clip(frames, params)
    e = vsa.Engine(max_streams=1, params=params)
    sid = e.stream_open(frames.shape[2], frames.shape[1], 8)
    for t in range(T):
        assert e.stream_push(sid, frames[t], pts=t) == 0
        if t == T - 1:
            e.stream_end(sid)
        e.step()
    _drain(e, [sid])
    _same(e.poll_frames(sid, 100), ref["frames"])
    _same_shots(e.poll_shots(sid, 100), ref["shots"])
    e.close()


def test_stream_without_frames(vsa, params):
    e = vsa.Engine(max_streams=2, params=params)
    sid = e.stream_open(320, 180, 8)
    e.stream_end(sid)
    _drain(e, [sid])
    assert len(e.poll_frames(sid, 10)) == 0
    assert len(e.poll_shots(sid, 10)) == 0
    e.close()


def test_10bit_samples_above_1023(vsa, params):
    """A 10-bit plane with a sample above 1023 is refused when the library
    copies it from host memory (stream push and clip run); read in place from
    device memory it is analysed without a fault (the working-level histogram
    keeps its bins below 1024) and the stream still ends normally."""
    import torch
    W, H = 640, 360
    ok = np.full((H, W), 500, np.uint16)
    bad = ok.copy()
    bad[100, 200] = 1024
    e = vsa.Engine(max_streams=2, params=params)
    sid = e.stream_open(W, H, 10)
    assert e.stream_push(sid, ok, pts=0) == 0
    e.step()
    assert e.stream_push(sid, bad, pts=1) == vsa.E_INVAL
    assert "1023" in vsa.last_error()
    # in place from device memory: values far outside the range, run to the end
    big = torch.from_numpy(np.full((H, W), 4000, np.int16)).to("cuda:0")
    sid2 = e.stream_open(W, H, 10)
    for t in range(4):
        assert e.stream_push_tensor(sid2, big, pts=t) == 0
        if t == 3:
            e.stream_end(sid2)
        e.step()
        e.sync()
    for _ in range(20):
        if e.stream_done(sid2):
            break
        e.step()
        e.sync()
    assert e.stream_done(sid2)
    assert len(e.poll_frames(sid2, 16)) == 4
    e.close()
    with vsa.Clip(W, H, bit_depth=10, chunk=4, params=params) as c:
        with pytest.raises(vsa.VsaError) as ei:
            c.run(np.stack([ok, bad]))
        assert ei.value.code == vsa.E_INVAL
        assert len(c.run(np.stack([ok, ok]))["frames"]) == 2
