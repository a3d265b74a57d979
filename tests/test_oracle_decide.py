"""Pins of the oracle's decision logic on injected measure sequences (CPU only).

The decisions are a pure function of the measures, so each case feeds
sequences whose outcome follows from the rules by hand: keyframe spacing in
closed form, a hardcut, a one-frame flash, a K-frame dissolve with a plateau,
the 3:2 pulldown cadence and its phase, field order from v1 vs v2, static
frames skipped, the analysis cap, and the end of the clip.
"""
import numpy as np
import pytest

F_KEY, F_START, F_TRANS, F_FIRED, F_ANALYZED = 16, 32, 8, 4, 64


def seq(T, k_max, a=0.3, swr=0.05):
    kw = k_max + 2
    s = {"act": np.full(T, a), "swr": np.full(T, swr), "static": np.zeros(T, np.uint8),
         "v": np.tile([0.1, 1.0, 1.0], (T, 1)), "F": np.full((T, kw), a), "S": np.full((T, kw), swr),
         "P": np.full((T, kw), a)}
    return s


def fix(s):
    s["F"][:, 1] = s["act"]
    s["S"][:, 1] = s["swr"]
    return s


def run(orc, params, s, **kw):
    p = dict(params, **kw)
    return orc.decide_injected(fix(s), p)


def test_keyframe_spacing_closed_form(orc, params):
    # ACT 0.5 every frame, theta_kf 3.0: the sum exceeds 3.0 after 7 frames
    # (6 * 0.5 = 3.0 is not > 3.0), so keyframes fall on 0, 7, 14, ...
    T = 60
    r = run(orc, params, seq(T, 4, a=0.5))
    kf = np.nonzero(r["frames"]["flags"] & F_KEY)[0]
    assert kf.tolist() == list(range(0, T, 7))
    assert len(r["shots"]) == 1 and r["shots"][0]["first"] == 0 and r["shots"][0]["last"] == T - 1


def test_hardcut(orc, params):
    # every K verifies with the same excess: the first (K = 1) is taken
    T, c = 80, 30
    s = seq(T, 4)
    s["act"][c] = 2.0
    s["F"][c, :] = 2.0
    s["S"][c, :] = 0.8
    s["swr"][c] = 0.8
    r = run(orc, params, s)
    f = r["frames"]
    assert f["boundary"][c + 1] == 1 and f["boundary_k"][c + 1] == 1
    assert f["flags"][c] & F_FIRED
    assert f["flags"][c + 1] & F_START and f["flags"][c + 1] & F_KEY
    assert np.count_nonzero(f["boundary"]) == 1
    sh = r["shots"]
    assert [(s_["first"], s_["last"]) for s_ in sh] == [(0, c), (c + 1, T - 1)]
    assert sh[1]["in_boundary"] == 1 and sh[1]["in_k"] == 1
    assert np.all(f["shot_id"][:c + 1] == 0) and np.all(f["shot_id"][c + 1:] == 1)


def test_one_frame_flash_is_not_a_boundary(orc, params):
    T, fl = 80, 30          # frame 30 is bright
    s = seq(T, 4)
    s["act"][fl - 1] = 2.0  # 29 -> 30
    s["act"][fl] = 2.0      # 30 -> 31
    s["F"][fl - 1, 2:] = 0.3   # 29 -> 31, 32, ... are ordinary
    s["P"][fl, 1] = 2.0        # 30 -> 29 is the flash again
    r = run(orc, params, s)
    f = r["frames"]
    assert np.count_nonzero(f["boundary"]) == 0
    assert f["flags"][fl - 1] & F_FIRED
    assert len(r["shots"]) == 1


def test_dissolve_plateau(orc, params):
    # A 3-frame dissolve after t while the shot drifts: the backward activity
    # P_K grows with the distance K, and so does the forward activity F_K
    # past the end of the transition.  The excess E_K = F_K - P_K climbs over
    # the transition and then stays flat; the plain dissimilarity S_K keeps
    # growing, so a plateau on S would pick K = 4.
    T, t = 90, 50
    s = seq(T, 4, a=0.2)
    s["act"][t] = 0.6
    s["F"][t, 1:6] = [0.6, 1.4, 2.2, 2.4, 2.6]          # K = 1..5
    s["P"][t, 1:6] = [0.2, 0.4, 0.6, 0.8, 1.0]
    s["S"][t, 1:6] = [0.1, 0.2, 0.4, 0.8, 0.9]
    s["swr"][t] = 0.1
    r = run(orc, params, s, rho_d=1.5, theta_d=0.4, gamma=0.8)
    f = r["frames"]
    # V_1: 0.6 > 0.7 fails; V_2..V_5 hold, so C = {2, 3, 4}; E = 1.0, 1.6, 1.6;
    # the first E >= 0.8 * 1.6 is K = 3
    assert f["boundary"][t + 3] == 2 and f["boundary_k"][t + 3] == 3
    assert np.all(f["flags"][t + 1:t + 3] & F_TRANS)
    assert np.all(f["shot_id"][t + 1:t + 3] == -1)
    assert r["shots"][1]["first"] == t + 3 and r["shots"][0]["last"] == t
    # gamma = 0 takes the shortest verified transition
    r0 = run(orc, params, s, rho_d=1.5, theta_d=0.4, gamma=0.0)
    assert r0["frames"]["boundary_k"][t + 2] == 2


def _sampling(orc, params, v_of_phase, T=40, **kw):
    s = seq(T, 4, a=0.3)
    for t in range(T):
        s["v"][t] = v_of_phase(t % 5)
    return run(orc, params, s, **kw)


def test_pulldown_cadence_and_phase(orc, params):
    def v(ph):   # phases 2 and 3 mix two film frames
        return [1.0, 1.2, 0.1] if ph in (2, 3) else [0.1, 1.0, 0.1 if ph == 1 else 1.0]
    r = _sampling(orc, params, v)
    sh = r["shots"][0]
    assert sh["sampling"] == 4 and sh["pulldown_phase"] == 2 and sh["n_analyzed"] == 20


@pytest.mark.parametrize("v,expect", [([0.5, 1.0, 0.5], 2), ([0.5, 0.5, 1.0], 3), ([0.1, 1.0, 1.0], 1)])
def test_field_order_and_progressive(orc, params, v, expect):
    r = _sampling(orc, params, lambda ph: v)
    assert r["shots"][0]["sampling"] == expect


def test_static_frames_not_analysed(orc, params):
    s = seq(40, 4)
    s["static"][:] = 1
    r = run(orc, params, s)
    assert r["shots"][0]["n_analyzed"] == 0 and r["shots"][0]["sampling"] == 0
    assert not np.any(r["frames"]["flags"] & F_ANALYZED)
    assert np.all(np.isnan(r["frames"]["v"]))


def test_analysis_cap(orc, params):
    r = run(orc, params, seq(200, 4), n_ss=17)
    assert r["shots"][0]["n_analyzed"] == 17
    assert np.count_nonzero(r["frames"]["flags"] & F_ANALYZED) == 17


@pytest.mark.parametrize("T", [1, 2, 3])
def test_short_clips(orc, params, T):
    r = run(orc, params, seq(T, 4))
    assert len(r["frames"]) == T and len(r["shots"]) == 1
    assert r["shots"][0]["last"] == T - 1
    assert r["frames"]["flags"][0] & F_KEY and r["frames"]["flags"][0] & F_START
    assert not (r["frames"]["flags"][T - 1] & 1)   # last frame has no pair


def test_dense_equals_sparse(orc, params):
    rng = np.random.default_rng(0)
    for _ in range(5):
        T = int(rng.integers(20, 150))
        s = seq(T, 4)
        s["act"] = rng.uniform(0.1, 0.6, T)
        s["act"][rng.integers(5, T - 5, 3)] = 2.0
        s["v"] = rng.uniform(0, 1, (T, 3))
        s["F"] = rng.uniform(0.2, 2.5, s["F"].shape)
        s["S"] = rng.uniform(0, 1, s["S"].shape)
        s["P"] = rng.uniform(0.1, 0.8, s["P"].shape)
        sp = run(orc, params, {k: v.copy() for k, v in s.items()})
        de = orc.decide_injected(fix(s), params, dense=True)
        for name in ("flags", "shot_id", "boundary", "boundary_k", "field_mask"):
            assert np.array_equal(sp["frames"][name], de["frames"][name])
        ks = {tuple(k) for k in sp["keys"].tolist()}
        kd = {tuple(k) for k in de["keys"].tolist()}
        assert ks <= kd and len(kd) > len(ks)
