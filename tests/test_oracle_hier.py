"""Pins of the oracle's coarse-to-fine motion field (search = 1; CPU only).

The reading (Sec. III.A motion field, hierarchical variant): I and J are
box-downscaled once; every whole 8x8 block of the coarse I gets its full-search
vector d_c in [-R, R]^2 against the coarse J; a block (bx, by) of I whose
coarse block (bx/2, by/2) is whole is predicted by 2 d_c, any other by (0, 0);
its vector is the best of prediction + e, e in [-r, r]^2, against J (clamp to
edge), ties by the order (|e|^2, ey, ex).  Pinned here by an exhaustive
search written from that definition on tiny inputs, by known translations
beyond the full search's reach recovered exactly, by the special case that
reduces to the (separately pinned) full search, and on whole clips by
generator truth.
"""
import numpy as np
import pytest

import synth


def box(a):
    """One 2x2 box step, rounding half up, trailing odd row/column dropped."""
    a = a.astype(np.int64)
    h, w = a.shape[0] // 2, a.shape[1] // 2
    s = a[0:2 * h:2, 0:2 * w:2] + a[1:2 * h:2, 0:2 * w:2] + a[0:2 * h:2, 1:2 * w:2] + a[1:2 * h:2, 1:2 * w:2]
    return (s + 2) >> 2


def best_around(I, J, x0, y0, cx, cy, R):
    """Best (sad, dx, dy) of the block at (x0, y0) over (cx, cy) + e, e in [-R, R]^2."""
    h, w = J.shape
    blk = I[y0:y0 + 8, x0:x0 + 8]
    best = None
    for _, ey, ex in sorted((ex * ex + ey * ey, ey, ex) for ey in range(-R, R + 1) for ex in range(-R, R + 1)):
        yy = np.clip(np.arange(y0, y0 + 8)[:, None] + cy + ey, 0, h - 1)
        xx = np.clip(np.arange(x0, x0 + 8)[None, :] + cx + ex, 0, w - 1)
        s = int(np.abs(blk - J[yy, xx]).sum())
        if best is None or s < best[0]:
            best = (s, cx + ex, cy + ey)
    return best


def brute_hier(I, J, R, r):
    I = I.astype(np.int64)
    J = J.astype(np.int64)
    h, w = I.shape
    Ic, Jc = box(I), box(J)
    nbxc, nbyc = Ic.shape[1] // 8, Ic.shape[0] // 8
    mv = np.zeros((h // 8, w // 8, 2), np.int8)
    sad = np.zeros((h // 8, w // 8), np.int64)
    for by in range(h // 8):
        for bx in range(w // 8):
            px = py = 0
            if bx // 2 < nbxc and by // 2 < nbyc:
                _, cdx, cdy = best_around(Ic, Jc, 8 * (bx // 2), 8 * (by // 2), 0, 0, R)
                px, py = 2 * cdx, 2 * cdy
            s, dx, dy = best_around(I, J, 8 * bx, 8 * by, px, py, r)
            mv[by, bx] = (dx, dy)
            sad[by, bx] = s
    return mv, sad


def moments(I, J, mv):
    h, w = I.shape
    I = I.astype(np.int64)
    J = J.astype(np.int64)
    out = np.zeros(5, np.int64)
    for by in range(h // 8):
        for bx in range(w // 8):
            dx, dy = int(mv[by, bx, 0]), int(mv[by, bx, 1])
            x = I[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
            yy = np.clip(np.arange(8 * by, 8 * by + 8)[:, None] + dy, 0, h - 1)
            xx = np.clip(np.arange(8 * bx, 8 * bx + 8)[None, :] + dx, 0, w - 1)
            y = J[yy, xx]
            out += [x.sum(), y.sum(), (x * x).sum(), (y * y).sum(), (x * y).sum()]
    return tuple(int(v) for v in out)


def hp(params, R, r):
    return dict(params, search=1, radius=R, refine=r)


@pytest.mark.parametrize("seed,kind,h,w", [(0, "random", 32, 40), (1, "binary", 32, 48), (2, "shift", 40, 48),
                                           (3, "smooth", 48, 56), (4, "random", 24, 44)])
def test_bruteforce_small(orc, params, seed, kind, h, w):
    """Exhaustive two-stage search on tiny planes (R = 2, r = 1): random,
    binary (zero samples, ties), a shift beyond R, smooth content, and odd
    block counts whose last block column or row has no whole coarse block."""
    rng = np.random.default_rng(seed)
    if kind == "random":
        I = rng.integers(0, 256, (h, w)); J = rng.integers(0, 256, (h, w))
    elif kind == "binary":
        I = rng.integers(0, 2, (h, w)) * 255; J = rng.integers(0, 2, (h, w)) * 255
    elif kind == "shift":
        I = rng.integers(0, 256, (h, w)); J = np.roll(np.roll(I, 3, 0), -5, 1)
    else:
        I = np.cumsum(np.cumsum(rng.integers(-3, 4, (h, w)), 0), 1) % 256
        J = np.roll(I, (2, -4), (0, 1))
    I = I.astype(np.uint16); J = J.astype(np.uint16)
    ref_mv, ref_sad = brute_hier(I, J, 2, 1)
    got = orc.pair(I, J, hp(params, 2, 1))
    assert np.array_equal(got["mv"], ref_mv)
    assert np.array_equal(got["sad"], ref_sad)
    assert (got["sx"], got["sy"], got["sxx"], got["syy"], got["sxy"]) == moments(I, J, ref_mv)
    d2 = ref_mv[..., 0].astype(np.int64) ** 2 + ref_mv[..., 1].astype(np.int64) ** 2
    import math
    assert got["a"] == sum(math.isqrt(65536 * int(v)) for v in d2.ravel())


def test_bruteforce_r8(orc, params):
    """The shapes the engine uses: R = 8 coarse, r = 1 refine, a 64 x 48 pair."""
    rng = np.random.default_rng(7)
    I = (np.cumsum(np.cumsum(rng.integers(-4, 5, (48, 64)), 0), 1) % 256).astype(np.uint16)
    J = np.roll(I, (-9, 11), (0, 1)).astype(np.uint16)
    J[::7] = rng.integers(0, 256, J[::7].shape)
    ref_mv, ref_sad = brute_hier(I, J, 8, 1)
    got = orc.pair(I, J, hp(params, 8, 1))
    assert np.array_equal(got["mv"], ref_mv)
    assert np.array_equal(got["sad"], ref_sad)


def _texture(seed, h, w):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.gen.texture(rng, 256, 3.0, 16, 235)[:h, :w].astype(np.uint16)


@pytest.mark.parametrize("d", [(-16, 6), (14, -8), (16, 16), (13, -11), (17, -15), (-17, 17), (9, 0)])
def test_translation_beyond_full_search(orc, params, d):
    """A smooth texture moved by d with |d| up to 2R + r = 17.  With both
    components even the coarse planes are the same texture moved by d/2, so
    every interior block finds d with SAD 0.  With an odd component the
    coarse move is half a pixel; the coarse vector is then the nearer integer
    on either side or, at a few blocks, off by one in the other axis too, so
    most interior blocks (here at least 95%) find d with SAD 0.  The full
    search (reach R = 8) finds d at none of them."""
    I = _texture(11, 160, 192)
    J = np.roll(I, (d[1], d[0]), (0, 1))          # J(p + d) = I(p)
    got = orc.pair(I, J, hp(params, 8, 1))
    full = orc.pair(I, J, dict(params, search=0, radius=8))
    inner = (slice(4, 160 // 8 - 4), slice(4, 192 // 8 - 4))
    hit = (got["mv"][inner][..., 0] == d[0]) & (got["mv"][inner][..., 1] == d[1])
    assert np.all(got["sad"][inner][hit] == 0)
    if d[0] % 2 == 0 and d[1] % 2 == 0:
        assert hit.all()
    else:
        assert hit.mean() >= 0.95
    fhit = (full["mv"][inner][..., 0] == d[0]) & (full["mv"][inner][..., 1] == d[1])
    assert not fhit.any()


@pytest.mark.parametrize("h,w", [(8, 8), (15, 40), (40, 15), (12, 12)])
@pytest.mark.parametrize("r", [1, 2, 3])
def test_no_coarse_block_is_full_search(orc, params, h, w, r):
    """A plane too small for one whole coarse block predicts (0, 0) everywhere,
    so the coarse-to-fine field is the full search of radius r."""
    rng = np.random.default_rng(h * 100 + w + r)
    I = rng.integers(0, 1024, (h, w)).astype(np.uint16)
    J = rng.integers(0, 1024, (h, w)).astype(np.uint16)
    a = orc.pair(I, J, hp(params, 8, r))
    b = orc.pair(I, J, dict(params, search=0, radius=r))
    for k in ("mv", "sad"):
        assert np.array_equal(a[k], b[k])
    for k in ("sx", "sy", "sxx", "syy", "sxy", "a", "ncc", "act"):
        assert a[k] == b[k]


def test_identical_planes(orc, params):
    I = _texture(3, 96, 128)
    got = orc.pair(I, I.copy(), hp(params, 8, 1))
    assert not got["mv"].any() and got["ncc"] == 1.0 and got["a"] == 0


def test_fast_pans_lower_in_shot_activity(orc, params):
    """A 320x180 clip whose pans (10-16 px per frame) exceed the full
    search's reach: the coarse-to-fine field tracks them, so the activity of
    consecutive frames inside a shot drops well below the full search's, and
    the hardcut (generator truth) is still found exactly."""
    spec = synth.make_c1(seed=9, T=48)
    rng = np.random.default_rng(9)
    for s in spec.shots:
        s.pan = [(int(rng.choice([-1, 1]) * rng.integers(10, 17)), int(rng.integers(-4, 5)))
                 for _ in range(s.length + 16)]
    frames = synth.render(spec)
    full = orc.run_clip(frames, dict(params, search=0))
    hier = orc.run_clip(frames, dict(params, search=1, refine=1))
    cut = spec.truth()["boundaries"][0][1]
    inside = [t for t in range(len(frames) - 1) if t != cut - 1]
    a_full = full["frames"]["act"][inside]
    a_hier = hier["frames"]["act"][inside]
    assert np.median(a_hier) < 0.5 * np.median(a_full)
    b = hier["frames"]["boundary"]
    assert list(np.nonzero(b)[0]) == [cut] and b[cut] == 1
