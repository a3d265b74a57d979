"""GPU parity: every HIP kernel and the full engine against the CPU oracle.

Integers (levels, motion vectors, SADs, moments, A), labels and flags must be
bit-exact; NCC within 1e-6 absolute (the finishing arithmetic is expected to be
bitwise identical, which test_finish_bitwise checks on its own).
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

NCC_TOL = 1e-6


def _rand_plane(rng, h, w, maxv=255, kind="random"):
    if kind == "random":
        return rng.integers(0, maxv + 1, size=(h, w)).astype(np.uint16)
    if kind == "smooth":
        y, x = np.mgrid[0:h, 0:w]
        base = (np.sin(x / 5.0 + rng.uniform(0, 6)) + np.cos(y / 7.0 + rng.uniform(0, 6))) * 0.25 + 0.5
        noise = rng.integers(-3, 4, size=(h, w))
        return np.clip(np.rint(base * maxv) + noise, 0, maxv).astype(np.uint16)
    if kind == "periodic":
        tile = rng.integers(0, maxv + 1, size=(4, 4))
        return np.tile(tile, (h // 4 + 1, w // 4 + 1))[:h, :w].astype(np.uint16)
    if kind == "flat":
        return np.full((h, w), rng.integers(0, maxv + 1), np.uint16)
    if kind == "zeros_ones":
        return (rng.integers(0, 2, size=(h, w)) * maxv).astype(np.uint16)
    raise ValueError(kind)


def _shifted(I, dx, dy, rng, maxv, noise=0):
    J = np.roll(np.roll(I.astype(np.int64), dy, axis=0), dx, axis=1)
    if noise:
        J = J + rng.integers(-noise, noise + 1, size=J.shape)
    return np.clip(J, 0, maxv).astype(np.uint16)


# ---------------------------------------------------------------- pyramid (K1)

@pytest.mark.parametrize("W,H,bits", [(320, 180, 8), (2048, 1080, 8), (720, 576, 8), (1280, 720, 8),
                                      (1920, 1080, 8), (3840, 2160, 10), (333, 211, 8), (1001, 77, 10),
                                      (64, 32, 8), (4099, 2051, 8)])
def test_levels_bitexact(vsa, orc, params, W, H, bits):
    print(f"levels {W}x{H} {bits}-bit", flush=True)
    rng = np.random.default_rng(W * 7 + H)
    maxv = (1 << bits) - 1
    Y = rng.integers(0, maxv + 1, size=(H, W)).astype(np.uint8 if bits == 8 else np.uint16)
    p = dict(params, k_max=15)
    ref = orc.levels(Y, p, bits=bits)
    g = orc.geometry(W, H, p)
    got = vsa.debug_levels(Y, p, bit_depth=bits)
    k = 0
    ltop = min(g["L"] + 4, g["Lcap"])
    for l in range(g["L"], ltop + 1):
        a = ref[("F", l)].ravel()
        assert np.array_equal(got[k:k + a.size], a), f"frame level {l}"
        k += a.size
    for f in ("U", "D"):
        a = ref[(f, g["Lf"])].ravel()
        assert np.array_equal(got[k:k + a.size], a), f"field {f}"
        k += a.size
    assert k == got.size


# ------------------------------------------------------------ pair (K2 + K3)

PAIR_CASES = [
    # (w, h, kind, dx, dy, noise)
    (64, 64, "random", 0, 0, 0),
    (64, 64, "smooth", 3, -2, 2),
    (72, 40, "smooth", -8, 8, 1),     # ragged tiles, extreme displacement
    (40, 24, "random", 5, 7, 0),
    (136, 80, "periodic", 1, 1, 0),   # ties everywhere
    (96, 96, "flat", 0, 0, 0),
    (88, 56, "zeros_ones", 2, -3, 0), # zero-valued samples
    (512, 270, "smooth", 6, -5, 3),   # a 2K working level
    (1024, 270, "smooth", -7, 4, 3),  # a 2K field level
    (45, 36, "smooth", 2, 2, 1),      # odd width
]


@pytest.mark.parametrize("bits", [8, 10])
@pytest.mark.parametrize("case", PAIR_CASES)
def test_pair_bitexact(vsa, orc, params, bits, case):
    w, h, kind, dx, dy, noise = case
    print(f"pair {case} {bits}-bit", flush=True)
    rng = np.random.default_rng(w * 131 + h + bits)
    maxv = (1 << bits) - 1
    I = _rand_plane(rng, h, w, maxv, kind)
    J = _shifted(I, dx, dy, rng, maxv, noise) if kind != "random" or (dx or dy) else _rand_plane(rng, h, w, maxv)
    ref = orc.pair(I, J, params)
    got = vsa.debug_pair(I, J, params, bit_depth=bits)
    assert np.array_equal(got["mv"], ref["mv"])
    assert np.array_equal(got["sad"], ref["sad"])
    for k in ("sx", "sy", "sxx", "syy", "sxy", "n", "a", "B", "static"):
        assert got[k] == ref[k], k
    assert abs(got["ncc"] - ref["ncc"]) <= NCC_TOL
    for k in ("ncc", "swr", "amm", "act"):
        assert got[k] == ref[k] or (math.isnan(got[k]) and math.isnan(ref[k])), k


@pytest.mark.parametrize("bits", [8, 10])
def test_pair_zero_mv(vsa, orc, params, bits):
    rng = np.random.default_rng(5 + bits)
    maxv = (1 << bits) - 1
    I = _rand_plane(rng, 48, 64, maxv, "smooth")
    J = _shifted(I, 3, 1, rng, maxv, 2)
    ref = orc.pair(I, J, params, force_zero_mv=True)
    got = vsa.debug_pair(I, J, params, bit_depth=bits, force_zero_mv=True)
    assert np.all(got["mv"] == 0)
    assert np.array_equal(got["sad"], ref["sad"])
    for k in ("sx", "sy", "sxx", "syy", "sxy", "a", "ncc", "act"):
        assert got[k] == ref[k], k


def test_finish_bitwise(vsa, orc, params):
    """The device finishing arithmetic (int64 covariance, IEEE double sqrt and
    division) reproduces the host bit for bit."""
    rng = np.random.default_rng(11)
    tuples = []
    for _ in range(20000):
        B = int(rng.integers(1, 5000))
        n = 64 * B
        x = rng.integers(0, 1024, size=8)
        sx = int(rng.integers(0, 1023 * n + 1))
        sy = int(rng.integers(0, 1023 * n + 1))
        # keep moments consistent enough to give |NCC| <= 1 most of the time
        sxx = max(sx * sx // n + int(rng.integers(0, 10 ** 7)), 0)
        syy = max(sy * sy // n + int(rng.integers(0, 10 ** 7)), 0)
        sxy = sx * sy // n + int(rng.integers(-10 ** 6, 10 ** 6))
        a = int(rng.integers(0, 2900 * B))
        tuples.append((sx, sy, sxx, syy, sxy, n, a, B))
        del x
    # edge cases: zero variance, negative covariance, identical, big values
    tuples += [(640, 640, 6400, 6400, 6400, 64, 0, 1), (0, 0, 0, 0, 0, 64, 0, 1),
               (640, 0, 6400, 0, 0, 64, 362, 1), (6400, 6400, 640000, 640000, 640000, 6400, 0, 100),
               (255 * 276480, 0, 255 * 255 * 276480, 0, 0, 276480, 0, 4320)]
    ints = np.array(tuples, np.int64)
    got = vsa.debug_finish(ints, params["a0"])
    ref = np.array([orc.finish(t, params["a0"]) for t in ints])
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


# ----------------------------------------------------------- decisions (K6)

def _random_sequence(rng, T, k_max, style):
    kw = k_max + 2
    act = rng.uniform(0.1, 0.5, T)
    if style == "cuts":
        for c in rng.choice(np.arange(3, T - 3), size=max(1, T // 40), replace=False):
            act[c] = rng.uniform(1.2, 2.5)
    swr = rng.uniform(0.0, 0.2, T)
    stat = (rng.random(T) < 0.15).astype(np.uint8)
    v = rng.uniform(0.05, 1.0, (T, 3))
    F = rng.uniform(0.2, 2.5, (T, kw))
    S = rng.uniform(0.0, 1.0, (T, kw))
    P = rng.uniform(0.1, 1.0, (T, kw))
    F[:, 1] = act
    S[:, 1] = swr
    return {"act": act, "swr": swr, "static": stat, "v": v, "F": F, "S": S, "P": P}


def _cmp_records(got, ref, check_pair=True):
    assert len(got) == len(ref)
    for name in ("flags", "shot_id", "boundary", "boundary_k", "field_mask"):
        assert np.array_equal(got[name], ref[name]), name
    assert np.array_equal(got["frame"], ref["frame"])
    vg, vr = got["v"], ref["v"]
    assert np.array_equal(np.isnan(vg), np.isnan(vr))
    assert np.array_equal(vg[~np.isnan(vg)], vr[~np.isnan(vr)])
    if check_pair:
        for name in ("mom", "n_pix", "amm_num", "n_blocks"):
            assert np.array_equal(got[name], ref[name]), name
        for name in ("h_mean", "h_std", "h_mad"):     # exact sums, one rounding each: bitwise
            assert np.array_equal(got[name].view(np.uint64), ref[name].view(np.uint64)), name
        for name in ("ncc", "swr", "amm", "act"):
            g, r = got[name], ref[name]
            assert np.array_equal(np.isnan(g), np.isnan(r)), name
            ok = ~np.isnan(r)
            assert np.all(np.abs(g[ok] - r[ok]) <= (NCC_TOL if name == "ncc" else 0.0)), name


def _cmp_shots(got, ref):
    assert len(got) == len(ref)
    for name in ("shot_id", "first", "last", "in_boundary", "in_k", "sampling", "pulldown_phase",
                 "n_analyzed", "final"):
        assert np.array_equal(got[name], ref[name]), name


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("dense", [False, True])
def test_decide_injected(vsa, orc, params, seed, dense):
    rng = np.random.default_rng(seed)
    k_max = [1, 2, 4, 8][seed % 4]
    p = dict(params, k_max=k_max, rho_f=float(rng.uniform(1.0, 3.0)), theta_f=float(rng.uniform(0.0, 0.3)),
             rho_d=float(rng.uniform(0.5, 3.0)), theta_d=float(rng.uniform(0.0, 0.5)),
             n_ss=int(rng.integers(5, 25)), theta_kf=float(rng.uniform(0.5, 4.0)))
    T = int(rng.integers(2, 300))
    seq = _random_sequence(rng, T, k_max, "cuts" if seed % 2 else "noise")
    ref = orc.decide_injected(seq, p, dense=dense)
    got = vsa.debug_decide(seq, p, dense=dense, k_max=k_max)
    _cmp_records(got["frames"], ref["frames"], check_pair=False)
    _cmp_shots(got["shots"], ref["shots"])
    rk = ref["keys"][ref["keys"]["kind"] != 0]
    assert np.array_equal(np.sort(got["keys"]), np.sort(rk))


def test_decide_pinned_branches(vsa, orc, params):
    """The hand-built sequences that pin the pass's rarer branches on the
    oracle (look-back truncated at the shot start, the clip end's missing
    V_{K+1}, the interlace vote's middle band, the field-order tie, a flash
    before a dissolve) give the same records, shots and measure requests on
    the device decision kernel."""
    import test_oracle_decide as tod
    for name, seq, kw in tod.branch_cases():
        p = dict(params, **kw)
        ref = orc.decide_injected(seq, p)
        got = vsa.debug_decide(seq, p, k_max=p["k_max"])
        _cmp_records(got["frames"], ref["frames"], check_pair=False)
        _cmp_shots(got["shots"], ref["shots"])
        rk = ref["keys"][ref["keys"]["kind"] != 0]
        assert np.array_equal(np.sort(got["keys"]), np.sort(rk)), name


# ------------------------------------------------------------- full engine

def _engine_vs_oracle(vsa, orc, params, frames, bits=8, dense=False, k_max=0):
    p = dict(params)
    if k_max:
        p["k_max"] = k_max
    ref = orc.run_clip(frames, p, bits=bits, dense=dense, want_mv=True)
    got = vsa.run_clip(frames, p, bit_depth=bits, dense=dense, debug_log=True, want_mv=True)
    _cmp_records(got["frames"], ref["frames"])
    _cmp_shots(got["shots"], ref["shots"])
    rk = ref["keys"][ref["keys"]["kind"] != 0]
    assert np.array_equal(np.sort(got["keys"]), np.sort(rk))
    assert np.array_equal(got["mv"], ref["mv"])
    return got, ref


def test_engine_c1(vsa, orc, params):
    spec = synth.make_c1()
    frames = synth.render(spec)
    print("engine C1", frames.shape, flush=True)
    _engine_vs_oracle(vsa, orc, params, frames)


def test_engine_c1_dense(vsa, orc, params):
    spec = synth.make_c1(T=24)
    frames = synth.render(spec)
    got, ref = _engine_vs_oracle(vsa, orc, params, frames, dense=True)
    sparse = orc.run_clip(frames, params)
    _cmp_records(got["frames"], sparse["frames"])


def test_engine_small_kmax8(vsa, orc, params):
    spec = synth.make_c2(seed=21, T=60, W=512, H=272, k_dis=8)
    frames = synth.render(spec)
    print("engine 512x272", frames.shape, flush=True)
    _engine_vs_oracle(vsa, orc, params, frames, k_max=8)


def test_engine_10bit(vsa, orc, params):
    spec = synth.make_c5(seed=9, T=16, W=640, H=360)
    frames = synth.render(spec)
    print("engine 10-bit", frames.shape, flush=True)
    _engine_vs_oracle(vsa, orc, params, frames, bits=10)


def test_engine_batched_mixed(vsa, orc, params):
    """Several streams of uneven shapes in one engine; each equals its oracle run."""
    clips = [synth.render(synth.make_c1(seed=31, T=20)),
             synth.render(synth.make_c2(seed=32, T=26, W=720, H=576)),
             synth.render(synth.make_c2(seed=33, T=14, W=1280, H=720))]
    refs = [orc.run_clip(c, params) for c in clips]
    e = vsa.Engine(max_streams=8, params=params)
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
        _cmp_records(e.poll_frames(s, 1000), r["frames"])
        _cmp_shots(e.poll_shots(s, 1000), r["shots"])
    e.close()


def test_engine_2k_bench_config(vsa, orc, params):
    """Full size, in the launch configuration the benchmark times: 256 streams
    of 2048x1080 8-bit in one engine, k_max 8, autotuned motion-search grids,
    the intensity measure on, frames borrowed from device memory.  Three
    sampled streams are compared record by record with the oracle on the same
    frame sequences (the oracle takes seconds per 2K stream)."""
    import torch
    import bench
    F, B, S = 96, 256, 40
    W, H = 2048, 1080
    frames = bench.render_frames(("c2", 2, 1500, W, H), F, W, H, 16)
    print("engine 2K x 64 streams", frames.shape, flush=True)
    dev = torch.from_numpy(frames).to("cuda:0")
    torch.cuda.synchronize()
    p = dict(params, k_max=8)
    e = vsa.Engine(max_streams=B, params=p)
    sids = np.array([e.stream_open(W, H, 8) for _ in range(B)], np.int32)
    offs = (np.arange(B) * 37) % F
    base = np.uint64(dev.data_ptr())
    pitches = np.full(B, W, np.int64)
    for s in range(S):
        ptrs = base + ((offs + s) % F).astype(np.uint64) * np.uint64(W * H)
        assert e.stream_push_batch(sids, ptrs, pitches, vsa.SRC_DEVICE_BORROW, None) == 0
        if s == S - 1:
            for sid in sids:
                e.stream_end(int(sid))
        e.step()
    guard = 0
    while not all(e.stream_done(int(sid)) for sid in sids):
        e.step()
        e.sync()
        guard += 1
        assert guard < 100
    for i in (0, 131, 255):
        seq = np.ascontiguousarray(frames[(offs[i] + np.arange(S)) % F])
        ref = orc.run_clip(seq, p)
        _cmp_records(e.poll_frames(int(sids[i]), 1000), ref["frames"])
        _cmp_shots(e.poll_shots(int(sids[i]), 1000), ref["shots"])
    e.close()


@pytest.mark.parametrize("wgs", [1, 3, 8])
def test_engine_fixed_launch_schedules(vsa, orc, params, wgs):
    """The motion-search launch schedule (persistent workgroups per CU, fixed
    or autotuned) changes no output: each equals the oracle."""
    frames = synth.render(synth.make_c2(seed=41, T=30, W=720, H=576))
    ref = orc.run_clip(frames, params)
    e = vsa.Engine(max_streams=2, params=params, me_wgs_per_cu=wgs)
    sid = e.stream_open(720, 576, 8)
    for t in range(len(frames)):
        assert e.stream_push(sid, frames[t], pts=t) == 0
        if t == len(frames) - 1:
            e.stream_end(sid)
        e.step()
    while not e.stream_done(sid):
        e.step()
        e.sync()
    _cmp_records(e.poll_frames(sid, 100), ref["frames"])
    _cmp_shots(e.poll_shots(sid, 100), ref["shots"])
    e.close()
