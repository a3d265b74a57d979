"""GPU parity of the engine and the offline clip form with the dense flow
(search = 2) against the oracle.

Every pair the pass measures (consecutive frame pairs, the three field pairs
of the interlace test, the deep-check pairs) takes the dense inverse search
flow measure.  The device evaluates it in IEEE double with every sum in the
oracle's order (patch sums as 64-trees, row sums and the rows' sums in runs
of 64, each a tree, added in order), so every record, NCC included, must
equal the oracle's bit for bit, and the shots and the measures the pass asks
for must be the oracle's.
"""
import numpy as np
import pytest

import synth
from test_gpu_parity import _cmp_records, _cmp_shots

pytestmark = pytest.mark.gpu


def fp(params, **kw):
    return dict(params, search=2, **kw)


def _bitwise(got, ref):
    for name in ("ncc", "swr", "amm", "act"):
        g, r = got[name], ref[name]
        assert np.array_equal(np.isnan(g), np.isnan(r)), name
        ok = ~np.isnan(r)
        assert np.array_equal(g[ok].view(np.uint64), r[ok].view(np.uint64)), name


def _flow_vs_oracle(vsa, orc, p, frames, bits=8, dense=False):
    ref = orc.run_clip(frames, p, bits=bits, dense=dense)
    got = vsa.run_clip(frames, p, bit_depth=bits, dense=dense, debug_log=True)
    _cmp_records(got["frames"], ref["frames"])
    _bitwise(got["frames"], ref["frames"])
    _cmp_shots(got["shots"], ref["shots"])
    rk = ref["keys"][ref["keys"]["kind"] != 0]
    assert np.array_equal(np.sort(got["keys"]), np.sort(rk))
    assert np.all(got["frames"]["n_blocks"] == 0) and np.all(got["frames"]["mom"] == 0)
    return got, ref


def test_flow_engine_c1(vsa, orc, params):
    frames = synth.render(synth.make_c1())
    print("dense flow engine C1", frames.shape, flush=True)
    got, _ = _flow_vs_oracle(vsa, orc, fp(params), frames)
    b = got["frames"]["boundary"]
    assert list(np.nonzero(b)[0]) == [32]


def test_flow_engine_dense(vsa, orc, params):
    frames = synth.render(synth.make_c1(T=24))
    print("dense flow engine C1, dense schedule", flush=True)
    _flow_vs_oracle(vsa, orc, fp(params), frames, dense=True)


def test_flow_engine_interlaced_mix(vsa, orc, params):
    """720x576 interlaced / pulldown content, k_max 8: the field pairs (the
    lower field read on the upper field's rows) take the flow too."""
    frames = synth.render(synth.make_mix_clip(0, seed=3, T=300), range(40))
    print("dense flow engine 720x576 mix, 40 frames", flush=True)
    got, ref = _flow_vs_oracle(vsa, orc, fp(params, k_max=8), frames)
    assert np.any(ref["keys"]["kind"] == 1)       # field pairs were measured


def test_flow_engine_10bit(vsa, orc, params):
    spec = synth.make_c5(seed=5, T=60, W=640, H=360)
    frames = synth.render(spec, range(20))
    print("dense flow engine 640x360 10-bit", flush=True)
    _flow_vs_oracle(vsa, orc, fp(params), frames, bits=10)


def test_flow_engine_2k(vsa, orc, params):
    """The 2K clip's first 24 frames (working level 512 x 270, field level
    1024 x 270, deep pairs down to 128 x 67) at k_max 8."""
    spec = synth.make_c2(seed=2, T=1500, W=2048, H=1080, k_dis=8)
    frames = synth.render(spec, range(24))
    print("dense flow engine 2K, 24 frames", flush=True)
    _flow_vs_oracle(vsa, orc, fp(params, k_max=8), frames)


def test_flow_engine_4k_10bit(vsa, orc, params):
    """3840 x 2160 10-bit 50i, 12 frames: working level 3 (480 x 270), field
    pairs at level 2 (960 x 540, the lower field read on the upper field's
    rows, weights 7 and 1 of the row and the row above, s = 3)."""
    spec = synth.make_c5(seed=7, T=60, W=3840, H=2160)
    frames = synth.render(spec, range(12))
    print("dense flow engine 4K 10-bit, 12 frames", flush=True)
    got, ref = _flow_vs_oracle(vsa, orc, fp(params), frames, bits=10)
    assert np.any(ref["keys"]["kind"] == 1)


def test_flow_engine_batched_mixed(vsa, orc, params):
    """Streams of uneven shapes in one engine (the scratch unit is the widest
    stream's); each equals its oracle run."""
    p = fp(params)
    clips = [synth.render(synth.make_c1(seed=31, T=20)),
             synth.render(synth.make_c2(seed=32, T=16, W=720, H=576)),
             synth.render(synth.make_c2(seed=33, T=10, W=1280, H=720))]
    refs = [orc.run_clip(c, p) for c in clips]
    e = vsa.Engine(max_streams=8, params=p)
    sids = [e.stream_open(c.shape[2], c.shape[1], 8) for c in clips]
    t = 0
    while not all(e.stream_done(s) for s in sids):
        for c, s in zip(clips, sids):
            if t < len(c):
                assert e.stream_push(s, c[t], pts=t) == 0
                if t == len(c) - 1:
                    e.stream_end(s)
        e.step()
        e.sync()
        t += 1
        assert t < 200
    for c, s, r in zip(clips, sids, refs):
        got = e.poll_frames(s, 1000)
        _cmp_records(got, r["frames"])
        _bitwise(got, r["frames"])
        _cmp_shots(e.poll_shots(s, 1000), r["shots"])
    with pytest.raises(vsa.VsaError):
        e.get_motion(sids[0], 0)                  # no block motion field with the flow
    e.close()


def test_flow_engine_open_later(vsa, orc, params):
    """A wider stream opened after a narrower one has run: the scratch grows
    between steps, both streams stay equal to their oracle runs."""
    p = fp(params)
    a = synth.render(synth.make_c1(seed=41, T=24))
    b = synth.render(synth.make_c2(seed=42, T=12, W=1280, H=720))
    ra, rb = orc.run_clip(a, p), orc.run_clip(b, p)
    e = vsa.Engine(max_streams=4, params=p)
    sa = e.stream_open(a.shape[2], a.shape[1], 8)
    sb = None
    t = 0
    while not (e.stream_done(sa) and sb is not None and e.stream_done(sb)):
        if t < len(a):
            assert e.stream_push(sa, a[t], pts=t) == 0
            if t == len(a) - 1:
                e.stream_end(sa)
        if t == 6:
            sb = e.stream_open(b.shape[2], b.shape[1], 8)
        if sb is not None and 0 <= t - 6 < len(b):
            assert e.stream_push(sb, b[t - 6], pts=t - 6) == 0
            if t - 6 == len(b) - 1:
                e.stream_end(sb)
        e.step()
        e.sync()                                  # collects the records, updates stream_done
        t += 1
        assert t < 200
    for s, r in ((sa, ra), (sb, rb)):
        got = e.poll_frames(s, 1000)
        _cmp_records(got, r["frames"])
        _bitwise(got, r["frames"])
        _cmp_shots(e.poll_shots(s, 1000), r["shots"])
    e.close()


_CLIP_REF = {}


@pytest.mark.parametrize("chunk", [7, 64])
def test_flow_clip_form(vsa, orc, params, chunk):
    frames = synth.render(synth.make_c1(seed=4, T=40))
    p = fp(params)
    if "c1" not in _CLIP_REF:
        _CLIP_REF["c1"] = orc.run_clip(frames, p)
    ref = _CLIP_REF["c1"]
    print(f"dense flow clip form, chunk {chunk}", flush=True)
    with vsa.Clip(320, 180, chunk=chunk, params=p, debug_log=True) as c:
        got = c.run(frames)
        log = c.measure_log()
    _cmp_records(got["frames"], ref["frames"])
    _bitwise(got["frames"], ref["frames"])
    _cmp_shots(got["shots"], ref["shots"])
    rk = ref["keys"][ref["keys"]["kind"] != 0]
    keys = np.zeros(len(log), rk.dtype)
    for i, name in enumerate(("kind", "ref", "oth", "ref_field", "oth_field", "level")):
        keys[name] = log[:, i]
    assert np.array_equal(np.sort(keys), np.sort(rk))


def test_flow_clip_interlaced_10bit(vsa, orc, params):
    """The clip form on 10-bit interlaced content (field pairs with the flow)."""
    frames = synth.render(synth.make_mix_clip(0, seed=3, T=300), range(32))
    frames10 = (frames.astype(np.uint16) * 4 + 1).astype(np.uint16)
    p = fp(params, k_max=8)
    ref = orc.run_clip(frames10, p, bits=10)
    with vsa.Clip(720, 576, chunk=16, params=p, bit_depth=10) as c:
        got = c.run(frames10)
    _cmp_records(got["frames"], ref["frames"])
    _bitwise(got["frames"], ref["frames"])
    _cmp_shots(got["shots"], ref["shots"])
