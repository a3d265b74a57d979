"""Pins of the oracle's dense inverse search flow (search = 2; CPU only).

The flow is an iterative estimate, so it is pinned by what the mathematics
fixes rather than by a second transcription: identical planes give zero flow
exactly; a two-dimensionally textured plane moved by an integer vector gives
that vector at every interior pixel (the search's fixed point, reached to
within 1e-3 px); a smooth analytic image moved by a sub-pixel vector gives it
to within the rounding of the samples; on a linear ramp (one gradient
direction everywhere) only the normal component of the motion is determined,
and the flow satisfies that component's constraint exactly; the measures
(NCC of I against J warped bilinearly by the flow, AMM = mean flow length)
equal scipy's bilinear resampling with clamped coordinates and numpy's Pearson
coefficient; whole clips keep the generator's hardcut.
"""
import numpy as np
import pytest

import synth


def fp(params):
    return dict(params, search=2)


def _texture(seed, size=256):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.gen.texture(rng, size, 3.0, 16, 235).astype(np.uint16)


def test_identical_planes_zero_flow(orc, params):
    I = _texture(1)[:64, :96]
    r = orc.flow_pair(I, I.copy(), fp(params))
    assert not r["flow"].any()
    assert r["ncc"] == 1.0 and r["amm"] == 0.0 and r["static"] == 1


@pytest.mark.parametrize("d", [(3, -2), (9, -4), (-6, 5), (0, 7), (1, 0)])
def test_integer_translation(orc, params, d):
    tex = _texture(11)
    I = tex[:96, :128]
    J = np.roll(tex, (d[1], d[0]), (0, 1))[:96, :128]        # J(p + d) = I(p)
    r = orc.flow_pair(I, J, fp(params))
    f = r["flow"][20:-20, 20:-20]
    assert np.abs(f[..., 0] - d[0]).max() < 1e-3
    assert np.abs(f[..., 1] - d[1]).max() < 1e-3


@pytest.mark.parametrize("d", [(3, -2), (-2, 4)])
def test_reverse_pair_opposite_flow(orc, params, d):
    tex = _texture(11)
    I = tex[:96, :128]
    J = np.roll(tex, (d[1], d[0]), (0, 1))[:96, :128]
    b = orc.flow_pair(J, I, fp(params))["flow"][20:-20, 20:-20]
    assert np.abs(b[..., 0] + d[0]).max() < 1e-3 and np.abs(b[..., 1] + d[1]).max() < 1e-3


def _field(x, y):
    return 120 + 40 * np.sin(x / 7.0) * np.cos(y / 9.0) + 30 * np.sin((x + 2 * y) / 11.0)


@pytest.mark.parametrize("d", [(1.5, -0.75), (4.25, 2.5), (-6.5, 3.0), (0.3, 0.2)])
def test_subpixel_translation(orc, params, d):
    """Samples of a smooth function and of the same function moved by d
    (both rounded to integers): the flow is d to within the rounding."""
    y, x = np.mgrid[0:96, 0:128].astype(np.float64)
    I = np.rint(_field(x, y)).astype(np.uint16)
    J = np.rint(_field(x - d[0], y - d[1])).astype(np.uint16)
    f = orc.flow_pair(I, J, fp(params))["flow"][16:-16, 16:-16]
    e = np.hypot(f[..., 0] - d[0], f[..., 1] - d[1])
    assert np.median(e) < 0.05 and np.percentile(e, 95) < 0.1


@pytest.mark.parametrize("d", [(3, -2), (-5, 1)])
def test_ramp_normal_flow(orc, params, d):
    """I = x + 2y: every patch sees the gradient g = (1, 2), so only g . u is
    observable; the flow meets g . (F - d) = 0 while its other component is
    left where the search started."""
    y, x = np.mgrid[0:48, 0:64]
    I = (x + 2 * y + 40).astype(np.uint16)
    J = (x - d[0] + 2 * (y - d[1]) + 40).astype(np.uint16)
    f = orc.flow_pair(I, J, fp(params))["flow"][16:-16, 16:-16]
    normal = (f[..., 0] - d[0]) + 2 * (f[..., 1] - d[1])
    assert np.abs(normal).max() < 1e-3


def test_measures_against_scipy(orc, params):
    from scipy.ndimage import map_coordinates
    tex = _texture(7)
    I = tex[:72, :104]
    J = np.roll(tex, (3, -5), (0, 1))[:72, :104].astype(np.int64)
    J = np.clip(J + np.random.default_rng(3).integers(-6, 7, J.shape), 0, 255).astype(np.uint16)
    r = orc.flow_pair(I, J, fp(params))
    F = r["flow"]
    yy, xx = np.mgrid[0:72, 0:104].astype(np.float64)
    Jw = map_coordinates(J.astype(np.float64), [yy + F[..., 1], xx + F[..., 0]], order=1, mode="nearest")
    ncc = np.corrcoef(I.astype(np.float64).ravel(), Jw.ravel())[0, 1]
    amm = np.hypot(F[..., 0], F[..., 1]).mean()
    assert abs(r["ncc"] - ncc) < 1e-12
    assert abs(r["amm"] - amm) < 1e-12
    assert abs(r["swr"] - (1.0 - r["ncc"])) == 0.0
    assert abs(r["act"] - np.sqrt((r["amm"] + params["a0"]) * r["swr"])) < 1e-15


def test_small_planes(orc, params):
    """Planes of one patch (8 x 8) up to a size with one coarser scale."""
    rng = np.random.default_rng(5)
    for h, w in ((8, 8), (8, 20), (15, 9), (17, 33)):
        I = rng.integers(0, 256, (h, w)).astype(np.uint16)
        r = orc.flow_pair(I, I.copy(), fp(params))
        assert not r["flow"].any() and r["ncc"] == 1.0
    with pytest.raises(ValueError):
        orc.flow_pair(np.zeros((7, 8), np.uint16), np.zeros((7, 8), np.uint16), fp(params))


def test_clip_hardcut(orc, params):
    """The 320x180 clip: the generator's hardcut at frame 32 (K = 1), both
    shots progressive, with the dense flow for every pair."""
    frames = synth.render(synth.make_c1(seed=1))
    r = orc.run_clip(frames, fp(params))
    b = r["frames"]["boundary"]
    assert list(np.nonzero(b)[0]) == [32] and b[32] == 1
    assert r["frames"]["boundary_k"][32] == 1
    assert list(r["shots"]["sampling"]) == [1, 1]
    assert np.all(r["frames"]["n_blocks"][:-1] == 0)      # no block field behind these records
