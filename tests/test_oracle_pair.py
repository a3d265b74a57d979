"""Pins of the oracle's pair measure (CPU only).

Motion field: exhaustive brute force on tiny inputs (written here from the
definition: full search, clamp-to-edge, tie order (|d|^2, dy, dx)), a known
translation, flat images, an explicit tie.  Moments/NCC: identities of the
normalised cross correlation (self-correlation 1, affine invariance, -1 for a
negated image, the Pearson coefficient of numpy), the zero-variance cases,
exact rational arithmetic within the rounding bound.  AMM: the fixed-point
mean of |d| from math.isqrt.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest


def brute_pair(I, J, R):
    """Exhaustive block search, written from the definition (slow, tiny inputs)."""
    h, w = I.shape
    I = I.astype(np.int64)
    J = J.astype(np.int64)
    cands = sorted(((dx * dx + dy * dy, dy, dx) for dy in range(-R, R + 1) for dx in range(-R, R + 1)))
    ys = np.arange(8)[:, None]
    xs = np.arange(8)[None, :]
    mv, sad = [], []
    for by in range(h // 8):
        for bx in range(w // 8):
            blk = I[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
            best = None
            for _, dy, dx in cands:   # first minimum in candidate order wins
                yy = np.clip(8 * by + ys + dy, 0, h - 1)
                xx = np.clip(8 * bx + xs + dx, 0, w - 1)
                s = int(np.abs(blk - J[yy, xx]).sum())
                if best is None or s < best[0]:
                    best = (s, dx, dy)
            mv.append((best[1], best[2]))
            sad.append(best[0])
    return np.array(mv, np.int8).reshape(h // 8, w // 8, 2), np.array(sad).reshape(h // 8, w // 8)


def warped_moments(I, J, mv):
    h, w = I.shape
    I = I.astype(np.int64)
    J = J.astype(np.int64)
    sx = sy = sxx = syy = sxy = 0
    for by in range(h // 8):
        for bx in range(w // 8):
            dx, dy = int(mv[by, bx, 0]), int(mv[by, bx, 1])
            x = I[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
            yy = np.clip(np.arange(8 * by, 8 * by + 8)[:, None] + dy, 0, h - 1)
            xx = np.clip(np.arange(8 * bx, 8 * bx + 8)[None, :] + dx, 0, w - 1)
            y = J[yy, xx]
            sx += int(x.sum()); sy += int(y.sum())
            sxx += int((x * x).sum()); syy += int((y * y).sum()); sxy += int((x * y).sum())
    return sx, sy, sxx, syy, sxy


@pytest.mark.parametrize("seed,kind", [(0, "random"), (1, "binary"), (2, "periodic"), (3, "shift")])
def test_bruteforce_r2(orc, params, seed, kind):
    rng = np.random.default_rng(seed)
    h, w = 24, 32
    if kind == "random":
        I = rng.integers(0, 256, (h, w)); J = rng.integers(0, 256, (h, w))
    elif kind == "binary":          # zero-valued samples and ties
        I = rng.integers(0, 2, (h, w)) * 255; J = rng.integers(0, 2, (h, w)) * 255
    elif kind == "periodic":
        t = rng.integers(0, 256, (2, 3))
        I = np.tile(t, (h // 2, w // 3 + 1))[:h, :w]; J = np.roll(I, 1, axis=1)
    else:
        I = rng.integers(0, 256, (h, w)); J = np.roll(np.roll(I, 1, 0), -2, 1)
    I = I.astype(np.uint16); J = J.astype(np.uint16)
    p = dict(params, radius=2)
    ref_mv, ref_sad = brute_pair(I, J, 2)
    got = orc.pair(I, J, p)
    assert np.array_equal(got["mv"], ref_mv)
    assert np.array_equal(got["sad"], ref_sad)
    assert (got["sx"], got["sy"], got["sxx"], got["syy"], got["sxy"]) == warped_moments(I, J, ref_mv)


def test_bruteforce_r8(orc, params):
    rng = np.random.default_rng(9)
    I = rng.integers(0, 256, (24, 24)).astype(np.uint16)
    J = np.clip(np.roll(I, (3, -5), (0, 1)).astype(int) + rng.integers(-4, 5, I.shape), 0, 255).astype(np.uint16)
    ref_mv, ref_sad = brute_pair(I, J, 8)
    got = orc.pair(I, J, params)
    assert np.array_equal(got["mv"], ref_mv)
    assert np.array_equal(got["sad"], ref_sad)


def test_known_translation(orc, params):
    rng = np.random.default_rng(5)
    big = rng.integers(0, 256, (200, 200)).astype(np.uint16)
    for vx, vy in [(3, -2), (-8, 8), (0, 5), (7, 0)]:
        I = big[50:114, 50:130]
        J = big[50 - vy:114 - vy, 50 - vx:130 - vx]   # content moves by +v
        got = orc.pair(I, J, params)
        nby, nbx = got["mv"].shape[:2]
        # blocks whose whole search window lies inside J
        for by in range(1, nby - 1):
            for bx in range(1, nbx - 1):
                assert tuple(got["mv"][by, bx]) == (vx, vy)
                assert got["sad"][by, bx] == 0


def test_flat_image_zero_motion(orc, params):
    I = np.full((40, 48), 77, np.uint16)
    J = np.full((40, 48), 77, np.uint16)
    got = orc.pair(I, J, params)
    assert np.all(got["mv"] == 0) and np.all(got["sad"] == 0)
    assert got["a"] == 0 and got["static"] == 1


def test_explicit_tie_order(orc, params):
    # checkerboard shifted by one pixel: every odd displacement has SAD 0; the
    # four of length 1 tie and (dx, dy) = (0, -1) comes first (smallest dy).
    y, x = np.mgrid[0:40, 0:40]
    I = ((x + y) % 2 * 200).astype(np.uint16)
    J = np.roll(I, 1, axis=1)
    got = orc.pair(I, J, params)
    assert tuple(got["mv"][2, 2]) == (0, -1)
    assert got["sad"][2, 2] == 0


def test_self_ncc_exactly_one(orc, params):
    rng = np.random.default_rng(1)
    for bits, maxv in ((8, 255), (10, 1023)):
        I = rng.integers(0, maxv + 1, (64, 96)).astype(np.uint16)
        got = orc.pair(I, I, params)
        assert got["ncc"] == 1.0 and got["swr"] == 0.0 and got["act"] == 0.0 and got["a"] == 0


@pytest.mark.parametrize("a,b", [(1, 0), (1, 17), (2, 3), (3, 1)])
def test_affine_brightness_invariance(orc, params, a, b):
    rng = np.random.default_rng(a * 10 + b)
    x = rng.integers(0, 80, (48, 64)).astype(np.int64)
    y = (a * x + b).astype(np.uint16)
    got = orc.pair(x.astype(np.uint16), y, params, force_zero_mv=True)
    if a == 1:
        assert got["ncc"] == 1.0
    else:
        assert abs(got["ncc"] - 1.0) <= 2 * np.finfo(float).eps


def test_negated_image(orc, params):
    rng = np.random.default_rng(2)
    x = rng.integers(0, 256, (48, 64))
    got = orc.pair(x.astype(np.uint16), (255 - x).astype(np.uint16), params, force_zero_mv=True)
    assert abs(got["ncc"] + 1.0) <= 2 * np.finfo(float).eps


def test_pearson(orc, params):
    rng = np.random.default_rng(3)
    for _ in range(5):
        x = rng.integers(0, 256, (40, 56))
        y = np.clip(x + rng.integers(-60, 61, x.shape), 0, 255)
        got = orc.pair(x.astype(np.uint16), y.astype(np.uint16), params, force_zero_mv=True)
        assert abs(got["ncc"] - np.corrcoef(x.ravel(), y.ravel())[0, 1]) <= 1e-12


def test_zero_variance_cases(orc, params):
    c = np.full((32, 32), 9, np.uint16)
    v = np.random.default_rng(4).integers(0, 256, (32, 32)).astype(np.uint16)
    assert orc.pair(c, c, params, force_zero_mv=True)["ncc"] == 1.0
    assert orc.pair(c, np.full((32, 32), 200, np.uint16), params, force_zero_mv=True)["ncc"] == 1.0
    assert orc.pair(c, v, params, force_zero_mv=True)["ncc"] == 0.0
    assert orc.pair(v, c, params, force_zero_mv=True)["ncc"] == 0.0


def test_amm_fixed_point(orc, params):
    rng = np.random.default_rng(6)
    I = rng.integers(0, 256, (64, 80)).astype(np.uint16)
    J = rng.integers(0, 256, (64, 80)).astype(np.uint16)
    got = orc.pair(I, J, params)
    mv = got["mv"].reshape(-1, 2).astype(int)
    A = sum(math.isqrt(65536 * (dx * dx + dy * dy)) for dx, dy in mv)
    assert got["a"] == A
    assert got["amm"] == A / (256.0 * got["B"])
    # floor(256 |d|) is within 1/256 px of |d| per block
    mags = np.sqrt((mv ** 2).sum(1))
    assert abs(got["a"] / 256.0 - mags.sum()) <= len(mags) / 256.0


def test_finish_against_exact_arithmetic(orc, params):
    getcontext().prec = 80
    rng = np.random.default_rng(7)
    ulp = np.finfo(float).eps
    for _ in range(300):
        B = int(rng.integers(1, 4000)); n = 64 * B
        x = rng.integers(0, 256, n); y = np.clip(x + rng.integers(-50, 51, n), 0, 255)
        sx, sy = int(x.sum()), int(y.sum())
        sxx, syy, sxy = int((x * x).sum()), int((y * y).sum()), int((x * y).sum())
        a = int(rng.integers(0, 2000 * B))
        ncc, swr, amm, act = orc.finish((sx, sy, sxx, syy, sxy, n, a, B), params["a0"])
        cov = n * sxy - sx * sy; vx = n * sxx - sx * sx; vy = n * syy - sy * sy
        exact = Decimal(cov) / (Decimal(vx) * Decimal(vy)).sqrt()
        assert abs(Decimal(ncc) - exact) <= Decimal(4 * ulp)
        assert swr == 1.0 - ncc
        assert abs(Decimal(amm) - Decimal(a) / Decimal(256 * B)) <= Decimal(ulp) * Decimal(amm)
        exact_act = ((Decimal(amm) + Decimal(params["a0"])) * Decimal(swr)).sqrt()
        assert abs(Decimal(act) - exact_act) <= Decimal(4 * ulp) * (exact_act + Decimal(1e-300))
