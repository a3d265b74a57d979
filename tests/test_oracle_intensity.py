"""Pins of the oracle's unary intensity measure H(t) (CPU only).

Sec. III.A lists the intensity histogram of a frame, with the mean, the
standard deviation and the mean absolute deviation taken from it.  The checks
are fixed by those definitions, not by the oracle's code: numpy's histogram,
mean, population standard deviation and mean absolute deviation about the
mean; closed forms for constant, two-valued and single-outlier images; the
exact integer sums by Python integers; shift and permutation invariance; and
the clip records, whose measures must be those of the frame's working-level
image.
"""
import math

import numpy as np
import pytest

import synth


def _numpy_measures(x):
    x = np.asarray(x, np.float64)
    mu = x.mean()
    return mu, x.std(), np.abs(x - mu).mean()


@pytest.mark.parametrize("bits,shape,seed", [(8, (37, 53), 0), (8, (1, 1), 1), (8, (270, 512), 2),
                                             (10, (64, 80), 3), (10, (135, 240), 4)])
def test_against_numpy(orc, bits, shape, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 1 << bits, shape)
    hist, ints, (mean, std, mad) = orc.intensity(x, bits)
    assert np.array_equal(hist, np.bincount(x.ravel(), minlength=1 << bits))
    m, s, d = _numpy_measures(x)
    assert math.isclose(mean, m, rel_tol=1e-13, abs_tol=1e-13)
    assert math.isclose(std, s, rel_tol=1e-12, abs_tol=1e-12)
    assert math.isclose(mad, d, rel_tol=1e-12, abs_tol=1e-12)


def test_exact_integer_sums(orc):
    rng = np.random.default_rng(7)
    x = rng.integers(0, 1024, (33, 47))
    _, ints, _ = orc.intensity(x, 10)
    v = [int(a) for a in x.ravel()]
    n, s1 = len(v), sum(v)
    assert ints["n"] == n
    assert ints["s1"] == s1
    assert ints["s2"] == sum(a * a for a in v)
    assert ints["m"] == sum(abs(n * a - s1) for a in v)


@pytest.mark.parametrize("c", [0, 17, 255])
def test_constant_image(orc, c):
    _, _, (mean, std, mad) = orc.intensity(np.full((20, 30), c), 8)
    assert (mean, std, mad) == (float(c), 0.0, 0.0)


@pytest.mark.parametrize("a,b", [(0, 255), (10, 20), (1023, 0)])
def test_two_values_half_and_half(orc, a, b):
    # N/2 pixels at a and N/2 at b: mean (a+b)/2, std = mad = |a-b|/2
    x = np.array([a, b] * 200).reshape(20, 20)
    bits = 10 if max(a, b) > 255 else 8
    _, _, (mean, std, mad) = orc.intensity(x, bits)
    assert mean == (a + b) / 2
    assert std == abs(a - b) / 2
    assert mad == abs(a - b) / 2


def test_single_outlier(orc):
    # N-1 zeros and one pixel at v: mean v/N, std v sqrt(N-1)/N, mad 2 v (N-1)/N^2
    n, v = 600, 200
    x = np.zeros(n, np.int64)
    x[123] = v
    _, _, (mean, std, mad) = orc.intensity(x.reshape(20, 30), 8)
    assert math.isclose(mean, v / n, rel_tol=1e-15)
    assert math.isclose(std, v * math.sqrt(n - 1) / n, rel_tol=1e-15)
    assert math.isclose(mad, 2 * v * (n - 1) / n ** 2, rel_tol=1e-15)


def test_shift_and_permutation_invariance(orc):
    rng = np.random.default_rng(11)
    x = rng.integers(0, 200, (24, 40))
    _, _, (m0, s0, d0) = orc.intensity(x, 8)
    _, _, (m1, s1, d1) = orc.intensity(x + 55, 8)
    assert (s1, d1) == (s0, d0)                 # exact sums: the numerators do not change
    assert math.isclose(m1, m0 + 55, rel_tol=1e-15)
    p = rng.permutation(x.ravel()).reshape(40, 24)
    assert orc.intensity(p, 8)[2] == (m0, s0, d0)


def test_rejects_out_of_range(orc):
    with pytest.raises(Exception):
        orc.intensity(np.full((4, 4), 256), 8)


def test_clip_records_use_the_working_level(orc, params):
    clip = synth.make_c1(seed=2)
    frames = synth.render(clip, range(12))
    res = orc.run_clip(frames, params)
    g = orc.geometry(frames.shape[2], frames.shape[1], params)
    for t in range(frames.shape[0]):
        work = orc.levels(frames[t], params)[("F", g["L"])]
        _, _, (mean, std, mad) = orc.intensity(work, 8)
        r = res["frames"][t]
        assert (r["h_mean"], r["h_std"], r["h_mad"]) == (mean, std, mad)
