"""GPU parity of the coarse-to-fine motion field (search = 1) against the oracle.

The coarse-to-fine kernel (16 x 16-block tiles: box-averaged coarse tile and
window in LDS, the full search's lane code on the coarse blocks, then a +-1
refinement per fine block around twice the coarse vector) must give the
oracle's motion vectors, SADs, moments and A bit for bit, and whole clips
the oracle's records, shots, measure keys and motion fields, through the
engine and the offline clip form.  Field pairs keep the full search in both.
"""
import math

import numpy as np
import pytest

import synth
from test_gpu_parity import NCC_TOL, _cmp_records, _cmp_shots, _engine_vs_oracle, _rand_plane, _shifted

pytestmark = pytest.mark.gpu

HIER_CASES = [
    # (w, h, kind, dx, dy, noise)
    (64, 48, "smooth", 9, -6, 1),      # one partial tile, beyond the full search's reach
    (40, 24, "random", 5, 7, 0),
    (136, 80, "periodic", 1, 1, 0),    # ties everywhere
    (200, 136, "smooth", -13, 11, 2),  # 25 x 17 blocks: the last block column and row have no coarse block
    (520, 280, "smooth", 16, -15, 2),  # a tile reaching past the row pitch
    (512, 270, "smooth", 12, 10, 3),   # a 2K working level
    (1024, 270, "smooth", -17, 3, 3),  # a 2K field-level shape, the reach's edge
    (88, 56, "zeros_ones", 2, -3, 0),  # zero-valued samples
    (96, 96, "flat", 0, 0, 0),
    (16, 16, "random", 1, 0, 0),       # one coarse block
    (15, 40, "random", 0, 2, 0),       # no whole coarse block: the refinement around (0, 0) alone
    (8, 8, "random", 0, 0, 0),
]


def _hp(params):
    return dict(params, search=1, refine=1)


@pytest.mark.parametrize("bits", [8, 10])
@pytest.mark.parametrize("case", HIER_CASES)
def test_hier_pair_bitexact(vsa, orc, params, bits, case):
    w, h, kind, dx, dy, noise = case
    print(f"coarse-to-fine pair {case} {bits}-bit", flush=True)
    rng = np.random.default_rng(w * 977 + h + bits)
    maxv = (1 << bits) - 1
    I = _rand_plane(rng, h, w, maxv, kind)
    J = _shifted(I, dx, dy, rng, maxv, noise) if kind != "random" or (dx or dy) else _rand_plane(rng, h, w, maxv)
    p = _hp(params)
    ref = orc.pair(I, J, p)
    got = vsa.debug_pair(I, J, p, bit_depth=bits)
    assert np.array_equal(got["mv"], ref["mv"])
    assert np.array_equal(got["sad"], ref["sad"])
    for k in ("sx", "sy", "sxx", "syy", "sxy", "n", "a", "B", "static"):
        assert got[k] == ref[k], k
    assert abs(got["ncc"] - ref["ncc"]) <= NCC_TOL
    for k in ("ncc", "swr", "amm", "act"):
        assert got[k] == ref[k] or (math.isnan(got[k]) and math.isnan(ref[k])), k


@pytest.mark.parametrize("bits", [8, 10])
def test_hier_pair_zero_mv(vsa, orc, params, bits):
    rng = np.random.default_rng(11 + bits)
    maxv = (1 << bits) - 1
    I = _rand_plane(rng, 136, 200, maxv, "smooth")
    J = _shifted(I, 3, 1, rng, maxv, 2)
    p = _hp(params)
    ref = orc.pair(I, J, p, force_zero_mv=True)
    got = vsa.debug_pair(I, J, p, bit_depth=bits, force_zero_mv=True)
    assert np.all(got["mv"] == 0)
    assert np.array_equal(got["sad"], ref["sad"])
    for k in ("sx", "sy", "sxx", "syy", "sxy", "a", "ncc", "act"):
        assert got[k] == ref[k], k


def _fast_pan_c1(seed, T, lo=10, hi=16):
    spec = synth.make_c1(seed=seed, T=T)
    rng = np.random.default_rng(seed)
    for s in spec.shots:
        s.pan = [(int(rng.choice([-1, 1]) * rng.integers(lo, hi + 1)), int(rng.integers(-4, 5)))
                 for _ in range(s.length + 16)]
    return spec


def test_hier_engine_c1(vsa, orc, params):
    frames = synth.render(synth.make_c1())
    print("coarse-to-fine engine C1", flush=True)
    _engine_vs_oracle(vsa, orc, _hp(params), frames)


def test_hier_engine_fast_pans_kmax8(vsa, orc, params):
    frames = synth.render(_fast_pan_c1(9, 64))
    print("coarse-to-fine engine, fast pans, k_max 8", flush=True)
    got, ref = _engine_vs_oracle(vsa, orc, _hp(params), frames, k_max=8)
    assert np.abs(got["mv"]).max() > 8          # vectors beyond the full search's reach


def test_hier_engine_dense(vsa, orc, params):
    frames = synth.render(synth.make_c1(T=24))
    _engine_vs_oracle(vsa, orc, _hp(params), frames, dense=True)


def test_hier_engine_10bit(vsa, orc, params):
    spec = synth.make_c5(seed=5, T=60, W=640, H=360)
    frames = synth.render(spec, range(36))
    print("coarse-to-fine engine 640x360 10-bit", flush=True)
    _engine_vs_oracle(vsa, orc, _hp(params), frames, bits=10)


def test_hier_engine_2k(vsa, orc, params):
    """The 2K clip's first 48 frames (working level 512 x 270, deep pairs up to
    level 5) at k_max 8."""
    spec = synth.make_c2(seed=2, T=1500, W=2048, H=1080, k_dis=8)
    frames = synth.render(spec, range(48))
    print("coarse-to-fine engine 2K, 48 frames", flush=True)
    _engine_vs_oracle(vsa, orc, _hp(params), frames, k_max=8)


def test_hier_engine_4k_10bit(vsa, orc, params):
    """3840 x 2160 10-bit: working level 3 (480 x 270), odd coarse block counts."""
    spec = synth.make_c5(seed=7, T=60, W=3840, H=2160)
    frames = synth.render(spec, range(20))
    print("coarse-to-fine engine 4K 10-bit, 20 frames", flush=True)
    _engine_vs_oracle(vsa, orc, _hp(params), frames, bits=10)


@pytest.mark.parametrize("chunk", [7, 64])
def test_hier_clip_form(vsa, orc, params, chunk):
    frames = synth.render(_fast_pan_c1(4, 64))
    p = _hp(params)
    ref = orc.run_clip(frames, p)
    with vsa.Clip(320, 180, chunk=chunk, params=p, debug_log=True) as c:
        got = c.run(frames)
        log = c.measure_log()
    _cmp_records(got["frames"], ref["frames"])
    _cmp_shots(got["shots"], ref["shots"])
    rk = ref["keys"][ref["keys"]["kind"] != 0]
    keys = np.zeros(len(log), rk.dtype)
    for i, name in enumerate(("kind", "ref", "oth", "ref_field", "oth_field", "level")):
        keys[name] = log[:, i]
    assert np.array_equal(np.sort(keys), np.sort(rk))


def test_hier_interlaced_mix_clip(vsa, orc, params):
    """720x576 interlaced / pulldown clip, k_max 8: field pairs full search,
    frame pairs coarse-to-fine, in the clip form."""
    p = dict(_hp(params), k_max=8)
    frames = synth.render(synth.make_mix_clip(0, seed=3, T=300), range(80))
    ref = orc.run_clip(frames, p)
    with vsa.Clip(720, 576, chunk=40, params=p) as c:
        got = c.run(frames)
    _cmp_records(got["frames"], ref["frames"])
    _cmp_shots(got["shots"], ref["shots"])
