"""End-to-end labels of the oracle against the generator's ground truth (CPU).

The truth comes from how the synthetic clips are built (where the cut is,
which frames are flashes, how each shot's fields were sampled), not from the
oracle.  The decision constants are the calibrated defaults; their values are
not fixed by the paper (parity unpinned as values), but these labels are what
the method is for: frame-accurate hardcuts, short dissolves, no boundary at a
flash (Sec. III.B), the sampling structure, field order and pulldown phase of
each shot (Sec. III.C), and a keyframe at every shot start (Sec. III.D).
"""
import numpy as np
import pytest

import synth

F_KEY = 16


@pytest.mark.parametrize("seed", range(6))
def test_c1_hardcut_and_progressive(orc, params, seed):
    # 64 frames of 320x180, iid motion in [-4, 4], hardcut 31 -> 32
    spec = synth.make_c1(seed=seed)
    tr = spec.truth()
    assert tr["boundaries"] == [(31, 32, 1)]
    r = orc.run_clip(synth.render(spec), params)
    f = r["frames"]
    b = np.nonzero(f["boundary"])[0].tolist()
    assert b == [32] and f["boundary"][32] == 1 and f["boundary_k"][32] == 1
    assert [(int(s["first"]), int(s["last"])) for s in r["shots"]] == [(0, 31), (32, 63)]
    assert all(int(s["sampling"]) == 1 for s in r["shots"])       # progressive
    kf = np.nonzero(f["flags"] & F_KEY)[0]
    assert 0 in kf and 32 in kf


@pytest.mark.slow
def test_2k_cut_dissolve_flashes_sampling(orc, params):
    # First 360 frames of a seeded 2048x1080 clip: progressive shot, hardcut
    # 108 -> 109, BFF interlaced shot, flashes at 148, 293, 303, 333 and 337,
    # a 4-frame dissolve 342 -> 346 into a 3:2 pulldown shot.
    spec = synth.make_c2(seed=13, T=600, W=2048, H=1080, k_dis=4)
    tr = spec.truth()
    assert tr["boundaries"] == [(108, 109, 1), (342, 346, 4)]
    n = 360
    rd = synth.Renderer(spec)
    frames = np.stack([rd.frame(t) for t in range(n)])
    r = orc.run_clip(frames, dict(params, k_max=4))
    f = r["frames"]
    got = [(int(t), int(f["boundary"][t])) for t in np.nonzero(f["boundary"])[0]]
    assert got[0] == (109, 1) and f["boundary_k"][109] == 1          # hardcut, frame-exact
    assert len(got) == 2 and got[1][1] == 2 and abs(got[1][0] - 346) <= 1   # dissolve, +-1 frame
    flashes = [x for x in spec.flashes if x < n]
    assert len(flashes) == 5
    for x in flashes:
        assert not np.any(f["boundary"][max(0, x - 1):x + 2])
    truth = {s["first"]: s for s in tr["shots"]}
    for s in r["shots"]:
        first = int(s["first"])
        t = truth.get(first) or truth.get(first + 1) or truth.get(first - 1)
        assert t is not None
        assert int(s["sampling"]) == t["sampling"]
        if t["sampling"] == 4:
            assert int(s["pulldown_phase"]) == t["pulldown_phase"]


@pytest.mark.slow
def test_8frame_dissolve_is_not_cut(orc, params):
    """Sec. III.B targets short dissolves (up to 4 frames); the 2K workload's
    8-frame linear dissolves are longer.  What the method does with one is
    pinned here: no boundary of either kind inside it or next to it (the fast
    check fires on three of its frames, and the deep check finds no K <= 8
    whose forward activity clearly exceeds the backward one), so the two shots
    are reported as one rather than cut in the middle.  Seed 3's dissolve,
    frames 558 -> 566, in a 68-frame window."""
    spec = synth.make_c2(seed=3, T=1500, W=2048, H=1080, k_dis=8)
    assert (558, 566, 8) in spec.truth()["boundaries"]
    a, b = 528, 596
    rd = synth.Renderer(spec)
    frames = np.stack([rd.frame(t) for t in range(a, b)])
    r = orc.run_clip(frames, dict(params, k_max=8))
    f = r["frames"]
    assert np.count_nonzero(f["boundary"]) == 0
    fired = (np.nonzero(f["flags"] & 4)[0] + a).tolist()
    assert any(558 <= t < 566 for t in fired)          # the deep check ran inside the dissolve
    assert len(r["shots"]) == 1
