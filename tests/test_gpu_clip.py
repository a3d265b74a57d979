"""Offline clip form (vsa_clip_*) against the oracle (GPU).

A clip taken `chunk` frames per launch must give the records and shots of the
oracle's sequential pass over the same frames: integers and labels exact,
doubles bitwise (the engine's kernels and finishing arithmetic are the same).
The sparse schedule computes some field measures speculatively (ahead of the
pass asking for them); records must still show exactly the ones it asked for.
Chunk sizes cover one frame, sizes that do not divide the clip (a ragged last
chunk), a chunk larger than the clip and the bench's 256; both schedules,
both sample widths, host and device sources, clips of 0-3 frames, and
repeated runs on one analyser.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

INT_FIELDS = ("frame", "flags", "shot_id", "boundary", "boundary_k", "field_mask", "mom", "n_pix", "amm_num",
              "n_blocks")
DBL_FIELDS = ("ncc", "swr", "amm", "act", "v", "h_mean", "h_std", "h_mad")


def _same(got, ref, what=""):
    gf, rf = got["frames"], ref["frames"]
    assert len(gf) == len(rf), what
    for name in INT_FIELDS:
        assert np.array_equal(gf[name], rf[name]), f"{what} {name}"
    for name in DBL_FIELDS:
        g, r = gf[name], rf[name]
        assert np.array_equal(np.isnan(g), np.isnan(r)), f"{what} {name} NaN pattern"
        ok = ~np.isnan(g)
        assert np.array_equal(g[ok].view(np.uint64), r[ok].view(np.uint64)), f"{what} {name}"
    gs, rs = got["shots"], ref["shots"]
    assert len(gs) == len(rs), f"{what} shots"
    for name in rs.dtype.names:
        assert np.array_equal(gs[name], rs[name]), f"{what} shot {name}"


def _same_requests(c, ref, what="", base=None):
    """The sparse measures the clip's sequential pass requested in its last
    run are the oracle's, as a set, and the counters (less `base`, the
    counters before that run) agree with them: every request was computed,
    as a regular task or speculatively ahead of the pass."""
    rk = ref["keys"][ref["keys"]["kind"] != 0]
    got = c.measure_log()
    keys = np.zeros(len(got), rk.dtype)
    for i, name in enumerate(("kind", "ref", "oth", "ref_field", "oth_field", "level")):
        keys[name] = got[:, i]
    assert np.array_equal(np.sort(keys), np.sort(rk)), f"{what} requested measures"
    cnt = c.counters()
    if base:
        cnt = {k: v - base[k] for k, v in cnt.items()}
    assert cnt["requested_measures"] == len(rk), what
    assert cnt["sparse_tasks"] >= cnt["requested_measures"], what
    # speculative tasks cover the field requests not computed as regular tasks
    assert cnt["speculative_tasks"] >= cnt["sparse_tasks"] - cnt["requested_measures"], what


def _n_chunks(T, C):
    """Chunks of a T-frame clip: a first one of min(C, max(16, C // 4)) frames, then C each."""
    head = min(C, max(16, C // 4))
    return 1 if T <= head else 1 + -(-(T - head) // C)


@pytest.fixture(scope="module")
def c1():
    return synth.render(synth.make_c1(seed=1))            # 320x180, 64 frames, a hardcut


@pytest.fixture(scope="module")
def c1_ref(orc, params, c1):
    return orc.run_clip(c1, params)


@pytest.mark.parametrize("chunk", [1, 7, 16, 64, 256])
def test_chunks_equal_oracle(vsa, params, c1, c1_ref, chunk):
    print(f"clip 320x180 chunk={chunk}", flush=True)
    with vsa.Clip(320, 180, chunk=chunk, params=params, debug_log=True) as c:
        got = c.run(c1)
        cnt = c.counters()
        _same_requests(c, c1_ref, f"chunk {chunk}")
    _same(got, c1_ref, f"chunk {chunk}")
    assert got["frames"]["pts"].tolist() == list(range(len(c1)))
    assert cnt["chunks"] == _n_chunks(len(c1), chunk)


def test_device_source_and_repeated_runs(vsa, orc, params, c1, c1_ref):
    import torch
    dev = torch.from_numpy(c1).to("cuda:0")
    with vsa.Clip(320, 180, chunk=16, params=params) as c:
        a = c.run_tensor(dev)
        b = c.run(c1[:40])                 # shorter clip on the same analyser
        d = c.run_tensor(dev)              # and the full one again
    _same(a, c1_ref, "device")
    _same(d, c1_ref, "device, third run")
    _same(b, orc.run_clip(c1[:40], params), "40 frames")


def test_strided_device_frames(vsa, orc, params, c1, c1_ref):
    """Frames laid out with a row pitch and a frame stride larger than needed."""
    import torch
    T, H, W = c1.shape
    big = torch.zeros((T, H + 3, W + 64), dtype=torch.uint8, device="cuda:0")
    big[:, :H, :W] = torch.from_numpy(c1).to("cuda:0")
    view = big[:, :H, :W]
    with vsa.Clip(W, H, chunk=24, params=params) as c:
        got = c.run_tensor(view)
    _same(got, c1_ref, "strided")


def test_dense_schedule(vsa, orc, params, c1):
    ref = orc.run_clip(c1, params, dense=True)
    with vsa.Clip(320, 180, chunk=16, dense=True, params=params) as c:
        got = c.run(c1)
    _same(got, ref, "dense")


def test_10bit(vsa, orc, params):
    c5 = synth.make_c5(seed=5, T=60, W=640, H=360)
    frames = synth.render(c5, range(40))
    ref = orc.run_clip(frames, params, bits=10)
    with vsa.Clip(640, 360, bit_depth=10, chunk=12, params=params) as c:
        got = c.run(frames)
    _same(got, ref, "10-bit")


def test_interlaced_mix_clip(vsa, orc, params):
    """720x576 clip with interlaced and pulldown shots, k_max 8."""
    p = dict(params)
    p["k_max"] = 8
    frames = synth.render(synth.make_mix_clip(0, seed=3, T=300), range(120))
    ref = orc.run_clip(frames, p)
    with vsa.Clip(720, 576, chunk=40, params=p, debug_log=True) as c:
        got = c.run(frames)
        _same_requests(c, ref, "720x576")
        # a second, shorter run logs only its own requests
        ref40 = orc.run_clip(frames[:40], p)
        base = c.counters()
        c.run(frames[:40])
        _same_requests(c, ref40, "720x576, 40 frames", base)
    _same(got, ref, "720x576")


def test_2k_bench_config(vsa, orc, params):
    """The 2048x1080 clip at the bench's chunk (256) and k_max (8), against
    the oracle on its first 160 frames (one ragged chunk) and the engine's
    stream form on 400 frames (a full chunk and a ragged one)."""
    import torch
    p = dict(params)
    p["k_max"] = 8
    spec = synth.make_c2(seed=2, T=1500, W=2048, H=1080, k_dis=8)
    frames = synth.render(spec, range(400))
    dev = torch.from_numpy(frames).to("cuda:0")
    with vsa.Clip(2048, 1080, chunk=256, params=p) as c:
        short = c.run_tensor(dev[:160])
        full = c.run_tensor(dev)
    _same(short, orc.run_clip(frames[:160], p), "2K, 160 frames")
    _same(full, vsa.run_clip(frames, p), "2K, 400 frames vs the stream form")


@pytest.mark.parametrize("T", [0, 1, 2, 3])
def test_short_clips(vsa, orc, params, T):
    frames = synth.render(synth.make_c1(seed=8, T=max(T, 2)), range(T)) if T else np.zeros((0, 180, 320), np.uint8)
    with vsa.Clip(320, 180, chunk=2, params=params) as c:
        got = c.run(frames)
    if T == 0:
        assert len(got["frames"]) == 0 and len(got["shots"]) == 0
        return
    _same(got, orc.run_clip(frames, params), f"{T} frames")


def test_run_argument_checks(vsa, params, c1):
    lib = vsa.lib()
    import ctypes as C
    with vsa.Clip(320, 180, chunk=8, params=params) as c:
        recs = np.zeros(4, vsa.FRAME_DTYPE)
        a = np.ascontiguousarray(c1[:4])
        p = a.ctypes.data_as(C.c_void_p)
        ns = C.c_int32(0)
        # pitch below a row, stride below a frame, device-copy source, negative count
        for stride, pitch, n, src in ((320 * 180, 319, 4, vsa.SRC_HOST), (320 * 179, 320, 4, vsa.SRC_HOST),
                                      (320 * 180, 320, 4, vsa.SRC_DEVICE_COPY), (320 * 180, 320, -1, vsa.SRC_HOST)):
            rc = lib.vsa_clip_run(c.h, p, stride, pitch, n, src, recs.ctypes.data_as(C.c_void_p), None, 0,
                                  C.byref(ns))
            assert rc == vsa.E_INVAL, (stride, pitch, n, src)
        # too few shot slots: the count is still reported
        rc = lib.vsa_clip_run(c.h, p, 320 * 180, 320, 4, vsa.SRC_HOST, recs.ctypes.data_as(C.c_void_p), None, 0,
                              C.byref(ns))
        assert rc == vsa.OK and ns.value >= 1
