"""Served form: each clip's results in a continuously batched mix equal its
results alone (GPU) and the oracle's sequential pass over the same frames.

Clips of different resolutions and bit depths arrive over time; the engine has
fewer stream slots and less HBM budget than the mix needs, so clips queue,
finished clips release their slots and memory, and later clips reuse them (a
reused slot must not see records or state of its previous stream).  Every
clip's per-frame records (integers, labels and doubles) and shot records must
be identical to a run of that clip alone through its own engine, and to the
oracle's records (integers and labels exact, NCC within 1e-6).  A run whose
per-step poll takes only a few records at a time must still deliver every
record of every clip.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

INT_FIELDS = ("frame", "flags", "shot_id", "boundary", "boundary_k", "mom", "n_pix", "amm_num", "n_blocks",
              "field_mask")
DBL_FIELDS = ("ncc", "swr", "amm", "act", "v", "h_mean", "h_std", "h_mad")


def _sources(torch):
    out = []
    out.append((synth.render(synth.make_c1(seed=1)), 8))                         # 320x180, 64 frames
    out.append((synth.render(synth.make_mix_clip(0, seed=3, T=300), range(40)), 8))   # 720x576 interlaced
    out.append((synth.render(synth.make_mix_clip(1, seed=3, T=300), range(40)), 8))   # 1280x720
    c5 = synth.make_c5(seed=5, T=60, W=640, H=360)
    out.append((synth.render(c5, range(48)), 10))                               # 640x360 10-bit
    return [(torch.from_numpy(a.astype(np.int16) if b == 10 else a).to("cuda:0"), a, b) for a, b in out]


def _compare(got, ref, cid):
    gf, rf = got.frames, ref["frames"]
    assert len(gf) == len(rf), f"clip {cid}: {len(gf)} vs {len(rf)} frame records"
    for name in INT_FIELDS:
        assert np.array_equal(gf[name], rf[name]), f"clip {cid}: {name}"
    for name in DBL_FIELDS:
        a, b = gf[name], rf[name]
        assert np.array_equal(np.isnan(a), np.isnan(b)), f"clip {cid}: {name} NaN pattern"
        ok = ~np.isnan(a)
        assert np.all(np.abs(a[ok] - b[ok]) <= 1e-6), f"clip {cid}: {name}"
    gs, rs = got.shots, ref["shots"]
    assert len(gs) == len(rs), f"clip {cid}: shots"
    for name in rs.dtype.names:
        assert np.array_equal(gs[name], rs[name]), f"clip {cid}: shot {name}"


@pytest.mark.parametrize("plain", [False, True])
def test_served_mix_equals_alone(vsa, orc, params, plain):
    import torch
    from paper_2502_09202_amd import serve
    print(f"served mix, plain={plain}", flush=True)
    src = _sources(torch)
    rng = np.random.default_rng(17)
    reqs = []
    for cid in range(12):
        s = cid % len(src)
        dev, host, bits = src[s]
        F = dev.shape[0]
        length = int(rng.integers(12, 90))
        start = int(rng.integers(0, F))
        arrival = 0.0 if cid < 10 else 0.01     # most at once (they must queue), two mid-flight
        reqs.append((serve.ClipRequest(cid, arrival, dev, start, length, bits), host))
    p = dict(params)
    # room for about three of the larger streams at once, and four slots
    big = vsa.Engine(max_streams=1, params=p)
    fp = max(big.footprint(h.shape[2], h.shape[1], r.bit_depth) for r, h in reqs)
    big.close()
    budget = int(3.5 * fp)
    S = serve.PlainServer if plain else serve.Server
    srv = S(max_streams=4, hbm_budget_bytes=budget, params=p)
    try:
        rep = srv.run([r for r, _ in reqs])
    finally:
        srv.close()
    assert len(rep.results) == len(reqs)
    assert rep.max_concurrent <= 4
    assert rep.refused_admissions > 0          # the mix did queue
    for r, host in reqs:
        frames = np.ascontiguousarray(host[(r.start + np.arange(r.length)) % host.shape[0]])
        ref = vsa.run_clip(frames, p, bit_depth=r.bit_depth)
        _compare(rep.results[r.cid], ref, r.cid)
        _compare(rep.results[r.cid], orc.run_clip(frames, p, bits=r.bit_depth), f"{r.cid} vs oracle")
    s = rep.summary()
    assert s["frames"] == sum(r.length for r, _ in reqs)
    assert s["frame_latency_ms_p99"] is not None and s["frame_latency_ms_p99"] >= s["frame_latency_ms_p50"]


def test_served_small_poll_cap_keeps_every_record(vsa, orc, params):
    """With a per-step poll of 3 records, 6 clips in flight publish more per
    step than one poll takes; a finished clip's queued records must be
    drained before its slot is freed."""
    import torch
    from paper_2502_09202_amd import serve
    host = synth.render(synth.make_c1(seed=1))
    dev = torch.from_numpy(host).to("cuda:0")
    reqs = [serve.ClipRequest(cid, 0.0, dev, 5 * cid, 30 + 3 * cid, 8) for cid in range(6)]
    srv = serve.Server(max_streams=8, params=params)
    try:
        rep = srv.run(reqs, poll_cap=3)
    finally:
        srv.close()
    assert len(rep.results) == len(reqs)
    assert rep.frames == sum(r.length for r in reqs)
    assert len(rep.frame_latency_ms) == rep.frames
    for r in reqs:
        frames = np.ascontiguousarray(host[(r.start + np.arange(r.length)) % host.shape[0]])
        _compare(rep.results[r.cid], orc.run_clip(frames, params), f"{r.cid} vs oracle")


def test_served_dense_flow_mix(vsa, orc, params):
    """The served form with the dense flow (search = 2): clips of four formats
    queue for three slots, finished clips release slots that later clips of
    other shapes reuse (sparse flow pairs planned for a closed stream are
    skipped, the flow scratch grows between steps), and every clip's records
    equal the oracle's, the measures bit for bit."""
    import torch
    from paper_2502_09202_amd import serve
    src = _sources(torch)
    rng = np.random.default_rng(23)
    reqs = []
    for cid in range(8):
        dev, host, bits = src[cid % len(src)]
        length = int(rng.integers(10, 24))
        start = int(rng.integers(0, dev.shape[0]))
        reqs.append((serve.ClipRequest(cid, 0.0 if cid < 6 else 0.01, dev, start, length, bits), host))
    p = dict(params, search=2)
    srv = serve.Server(max_streams=3, params=p)
    try:
        rep = srv.run([r for r, _ in reqs])
    finally:
        srv.close()
    assert len(rep.results) == len(reqs)
    assert rep.max_concurrent <= 3
    for r, host in reqs:
        frames = np.ascontiguousarray(host[(r.start + np.arange(r.length)) % host.shape[0]])
        ref = orc.run_clip(frames, p, bits=r.bit_depth)
        got = rep.results[r.cid]
        _compare(got, ref, f"{r.cid} vs oracle")
        for name in ("ncc", "swr", "amm", "act"):
            a, b = got.frames[name], ref["frames"][name]
            ok = ~np.isnan(b)
            assert np.array_equal(a[ok].view(np.uint64), b[ok].view(np.uint64)), f"clip {r.cid}: {name}"
