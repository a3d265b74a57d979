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


# ---------------------------------------------------------------------------
# Branches of the sequential pass that the cases above never reach.  Each
# expected outcome is worked out by hand from the rules (Sec. III.B-C as read
# in the design notes: R9-R11, R13, R14, R19); each fails if its branch is
# altered.

def _keys(r, kind):
    k = r["keys"]
    k = k[k["kind"] == kind]
    return sorted((int(a), int(b), int(c)) for a, b, c in zip(k["ref"], k["oth"], k["level"]))


def test_deep_check_at_shot_start_uses_no_lookback(orc, params):
    """Sec. III.B at t = shot start: K' = min(K, t - shot_start) = 0 for every
    K, so P_K = 0 and V_K <=> F_K > theta_d.  F_K = 1.0 > 0.4 everywhere: every
    K verifies with excess 1.0 and K* = 1.  No backward pair is measured; the
    huge P table would veto every K if it were read."""
    T = 30
    s = seq(T, 4, a=0.2)
    s["act"][0] = 2.0                   # fires against theta_f0 = 1.0 (no history)
    s["F"][0, :] = 1.0
    s["P"][0, :] = 100.0
    r = run(orc, params, s)
    f = r["frames"]
    assert f["flags"][0] & F_FIRED
    assert f["boundary"][1] == 1 and f["boundary_k"][1] == 1
    assert np.count_nonzero(f["boundary"]) == 1
    assert _keys(r, 3) == []                                  # no P_K requested
    assert _keys(r, 2) == [(0, 2, 1), (0, 3, 2), (0, 4, 2), (0, 5, 3)]   # F_K at levels ceil(log2 K)


def test_deep_check_truncated_lookback(orc, params):
    """Fast check firing 2 frames after the shot start (k_max 4): K' =
    min(K, 2), so the backward pairs are t -> t-1 (K = 1, level 0), then
    t -> t-2 at the levels of K = 2 (1), K = 3 and 4 (both 2, one measure) and
    K = 5 (3)."""
    T, t = 30, 2
    s = seq(T, 4, a=0.2)
    s["act"][t] = 2.0                   # history (0.2, 0.2): threshold 1.5 * 0.2 + 0.05 = 0.35
    s["F"][t, :] = 2.0
    s["P"][t, :] = 0.2
    r = run(orc, params, s)
    assert r["frames"]["flags"][t] & F_FIRED
    assert _keys(r, 3) == [(t, 0, 1), (t, 0, 2), (t, 0, 3), (t, 1, 0)]
    # every K verifies with the same excess 1.8: K* = 1
    assert r["frames"]["boundary"][t + 1] == 1


def test_deep_check_at_clip_end_takes_missing_next_as_true(orc, params):
    """Sec. III.B at the end of the clip: a fire at t = T - 2 can test only
    K = 1, and V_2 (no frame t + 2) counts as true, so the last frame starts a
    shot; at t = T - 3 with V_1 false and V_2 true, K = 2 is accepted with V_3
    missing: a 2-frame dissolve ending on the last frame."""
    T = 30
    s = seq(T, 4, a=0.2)
    s["act"][T - 2] = 2.0
    s["F"][T - 2, :] = 2.0
    s["P"][T - 2, :] = 0.2
    r = run(orc, params, s)
    f = r["frames"]
    assert f["boundary"][T - 1] == 1 and f["boundary_k"][T - 1] == 1
    assert [(int(x["first"]), int(x["last"])) for x in r["shots"]] == [(0, T - 2), (T - 1, T - 1)]

    s = seq(T, 4, a=0.2)
    s["act"][T - 3] = 0.5               # fires (threshold 0.35) but V_1: 0.5 > 1.3 * 0.2 + 0.4 = 0.66 fails
    s["F"][T - 3, 2:] = 2.0             # V_2: 2.0 > 0.66
    s["P"][T - 3, :] = 0.2
    r = run(orc, params, s)
    f = r["frames"]
    assert f["flags"][T - 3] & F_FIRED
    assert f["boundary"][T - 1] == 2 and f["boundary_k"][T - 1] == 2
    assert f["flags"][T - 2] & F_TRANS
    assert [(int(x["first"]), int(x["last"])) for x in r["shots"]] == [(0, T - 3), (T - 1, T - 1)]


def _analysed_shot(orc, params, v_rows, n_ss):
    """One shot whose first len(v_rows) frames are analysed with the given
    (v0, v1, v2); returns its shot record."""
    T = len(v_rows) + 5
    s = seq(T, 4, a=0.2)
    s["v"][:len(v_rows)] = np.array(v_rows, np.float64)
    r = run(orc, params, s, n_ss=n_ss)
    assert len(r["shots"]) == 1
    assert np.count_nonzero(r["frames"]["flags"] & F_ANALYZED) == len(v_rows)
    return r["shots"][0]


COMBED, PLAIN = (1.0, 0.75, 0.5), (0.1, 0.75, 0.5)     # v0 > 0.65 min(v1, v2) or not; v1 > v2


@pytest.mark.parametrize("combed_at,expect", [
    ((0, 1, 2, 5, 6, 7), 2),     # 6 of 10 in (eps n, (1 - eps) n): majority 6 > 5, interlaced; v1 > v2: TFF
    ((0, 2, 5, 7), 1),           # 4 of 10 in the band: 8 > 10 fails, progressive
    ((0, 2, 5, 6, 7), 1),        # 5 of 10: a tie is not a majority, progressive
    ((0, 5), 1),                 # 2 <= eps n = 2: progressive without the vote
    ((0, 1, 2, 3, 5, 6, 7, 8), 2),   # 8 >= (1 - eps) n = 8: interlaced without the vote
])
def test_interlace_vote_middle_band(orc, params, combed_at, expect):
    """Sec. III.C: the combed fraction strictly between eps and 1 - eps is
    decided by the majority (eps 0.2, 10 analysed frames).  The combed frames
    never sit at two neighbouring positions of the 5-frame unit alone, so the
    pulldown test does not apply."""
    rows = [COMBED if i in combed_at else PLAIN for i in range(10)]
    sh = _analysed_shot(orc, params, rows, 10)
    assert sh["n_analyzed"] == 10
    assert sh["sampling"] == expect


@pytest.mark.parametrize("rows,expect", [
    ([(1.0, 0.75, 0.5)] * 5 + [(1.0, 0.5, 0.625)] * 5, 2),    # s = 0; sum v1 6.25 > 5.625: TFF
    ([(1.0, 0.5, 0.75)] * 5 + [(1.0, 0.625, 0.5)] * 5, 3),    # s = 0; sum v1 5.625 < 6.25: BFF
    ([(1.0, 0.75, 0.5)] * 5 + [(1.0, 0.5, 0.75)] * 5, 2),     # s = 0; sums equal (6.25): TFF
])
def test_field_order_tie(orc, params, rows, expect):
    """Sec. III.C field order as the vote of beta = v1 / v2: with as many
    frames v1 > v2 as v1 < v2 (s = 0) the sums decide, TFF iff sum v1 >= sum v2
    (dyadic values, so the sums are exact)."""
    sh = _analysed_shot(orc, params, rows, 10)
    assert sh["sampling"] == expect


def test_flash_does_not_mask_a_following_dissolve(orc, params):
    """R9: a fired frame enters the fast-check history capped at its
    threshold.  Activity 0.2 for 10 frames (threshold 0.35), a flash at 10
    (3.0, fires, deep check rejects it: only K = 1 verifies), then a dissolve
    from 12 with activity 0.6.  With the cap the history mean is
    (7 * 0.2 + 0.35) / 8 = 0.21875, threshold 0.378125 < 0.6: it fires and the
    deep check finds K = 3 (excess 0.5, 0.8, 1.9, 2.0; first >= 0.5 * 2.0).
    With the flash's own 3.0 in the history the threshold would be 0.875 and
    the dissolve would pass unseen."""
    T = 40
    s = seq(T, 4, a=0.2)
    s["P"][:, :] = 0.1
    s["act"][10] = 3.0
    s["F"][10, 2:] = 0.3          # V_2 false: 0.3 < 1.3 * 0.1 + 0.4
    s["act"][12] = 0.6
    s["F"][12, 2:] = [1.2 - 0.3, 2.0, 2.1, 2.1]     # F_2 0.9, F_3 2.0, F_4 2.1, F_5 2.1
    r = run(orc, params, s)
    f = r["frames"]
    assert f["flags"][10] & F_FIRED and f["flags"][12] & F_FIRED
    assert f["boundary"][10 + 1] == 0
    assert f["boundary"][15] == 2 and f["boundary_k"][15] == 3
    assert np.count_nonzero(f["boundary"]) == 1


def branch_cases():
    """The hand-built sequences above as (name, sequence, parameter
    overrides), for running the device decision kernel on them too."""
    out = []
    T = 30
    s = seq(T, 4, a=0.2); s["act"][0] = 2.0; s["F"][0, :] = 1.0; s["P"][0, :] = 100.0
    out.append(("shot_start", s, {}))
    s = seq(T, 4, a=0.2); s["act"][2] = 2.0; s["F"][2, :] = 2.0; s["P"][2, :] = 0.2
    out.append(("truncated_lookback", s, {}))
    s = seq(T, 4, a=0.2); s["act"][T - 2] = 2.0; s["F"][T - 2, :] = 2.0; s["P"][T - 2, :] = 0.2
    out.append(("clip_end_k1", s, {}))
    s = seq(T, 4, a=0.2); s["act"][T - 3] = 0.5; s["F"][T - 3, 2:] = 2.0; s["P"][T - 3, :] = 0.2
    out.append(("clip_end_k2", s, {}))
    for i, combed_at in enumerate(((0, 1, 2, 5, 6, 7), (0, 2, 5, 7), (0, 2, 5, 6, 7))):
        s = seq(15, 4, a=0.2)
        s["v"][:10] = np.array([COMBED if j in combed_at else PLAIN for j in range(10)])
        out.append((f"vote_band_{i}", s, {"n_ss": 10}))
    for i, rows in enumerate(([(1.0, 0.75, 0.5)] * 5 + [(1.0, 0.5, 0.625)] * 5,
                              [(1.0, 0.5, 0.75)] * 5 + [(1.0, 0.625, 0.5)] * 5,
                              [(1.0, 0.75, 0.5)] * 5 + [(1.0, 0.5, 0.75)] * 5)):
        s = seq(15, 4, a=0.2)
        s["v"][:10] = np.array(rows)
        out.append((f"field_order_tie_{i}", s, {"n_ss": 10}))
    s = seq(40, 4, a=0.2); s["P"][:, :] = 0.1; s["act"][10] = 3.0; s["F"][10, 2:] = 0.3
    s["act"][12] = 0.6; s["F"][12, 2:] = [0.9, 2.0, 2.1, 2.1]
    out.append(("flash_then_dissolve", s, {}))
    return [(n, fix(s_), kw) for n, s_, kw in out]
