"""Pins of the oracle's pyramid and fields (CPU only).

Each check is fixed by the definition itself (2x2 box average rounded half up,
applied per level; fields = alternate rows, Sec. III.C), not by re-running the
oracle's own code: constant images, a checkerboard, a tile where per-level
rounding and a single 4x4 mean differ, the interleave identity, and the level
sizes floor-halving gives for the workload formats.
"""
import numpy as np
import pytest


def test_constant_image_stays_constant(orc, params):
    for v in (0, 1, 128, 255):
        Y = np.full((180, 320), v, np.uint8)
        lv = orc.levels(Y, params)
        for k, a in lv.items():
            assert np.all(a == v), k


def test_constant_10bit(orc, params):
    Y = np.full((270, 480), 1023, np.uint16)
    for a in orc.levels(Y, params, bits=10).values():
        assert np.all(a == 1023)


def test_checkerboard_2x2(orc):
    # 0/255 alternating pixels: every 2x2 box sums to 510 -> (510 + 2) >> 2 = 128
    y, x = np.mgrid[0:8, 0:8]
    img = ((x + y) % 2 * 255).astype(np.uint16)
    d = orc.downscale(img)
    assert d.shape == (4, 4) and np.all(d == 128)


def test_rounding_half_up(orc):
    # sums 2 -> (2+2)>>2 = 1 (half rounds up); sum 1 -> 0; sum 6 -> 2
    a = np.array([[1, 1], [0, 0]], np.uint16)
    assert orc.downscale(a)[0, 0] == 1
    a = np.array([[1, 0], [0, 0]], np.uint16)
    assert orc.downscale(a)[0, 0] == 0
    a = np.array([[3, 3], [0, 0]], np.uint16)
    assert orc.downscale(a)[0, 0] == 2


def test_two_step_rounding_differs_from_one_step(orc):
    # 4x4 tile whose 2x2 quads sum to 2, 2, 2, 0: per-level rounding gives
    # level-1 values 1, 1, 1, 0 and level 2 = (3 + 2) >> 2 = 1, while one
    # 4x4 mean would give (6 + 8) >> 4 = 0.
    t = np.array([[1, 1, 1, 1],
                  [0, 0, 0, 0],
                  [1, 1, 0, 0],
                  [0, 0, 0, 0]], np.uint16)
    l1 = orc.downscale(t)
    assert l1.tolist() == [[1, 1], [1, 0]]
    assert orc.downscale(l1)[0, 0] == 1


def test_odd_trailing_row_and_column_dropped(orc):
    a = np.arange(5 * 7, dtype=np.uint16).reshape(5, 7)
    d = orc.downscale(a)
    assert d.shape == (2, 3)
    # top-left box is [[0,1],[7,8]] -> (16+2)>>2 = 4
    assert d[0, 0] == 4


def test_fields_interleave_restore_frame(orc, params):
    # L = 0 (width <= wmax): the field level is 0, so U and D are the rows themselves
    rng = np.random.default_rng(3)
    Y = rng.integers(0, 256, size=(180, 320)).astype(np.uint8)
    lv = orc.levels(Y, params)
    g = orc.geometry(320, 180, params)
    assert g["Lf"] == 0
    U, D = lv[("U", 0)], lv[("D", 0)]
    back = np.empty((180, 320), np.uint16)
    back[0::2] = U
    back[1::2] = D
    assert np.array_equal(back, Y)
    assert np.array_equal(lv[("F", 0)], Y)


def test_field_level_is_box_of_alternate_rows(orc, params):
    # 2K: Lf = 1, so U_1[y][x] = box of rows 4y and 4y+2 (the even rows), columns 2x, 2x+1
    rng = np.random.default_rng(4)
    Y = rng.integers(0, 256, size=(1080, 2048)).astype(np.uint8)
    lv = orc.levels(Y, params)
    U = lv[("U", 1)].astype(np.int64)
    D = lv[("D", 1)].astype(np.int64)
    Yi = Y.astype(np.int64)
    for (yy, xx) in [(0, 0), (5, 17), (269, 1023), (100, 500)]:
        s = Yi[4 * yy, 2 * xx] + Yi[4 * yy, 2 * xx + 1] + Yi[4 * yy + 2, 2 * xx] + Yi[4 * yy + 2, 2 * xx + 1]
        assert U[yy, xx] == (s + 2) >> 2
        s = Yi[4 * yy + 1, 2 * xx] + Yi[4 * yy + 1, 2 * xx + 1] + Yi[4 * yy + 3, 2 * xx] + Yi[4 * yy + 3, 2 * xx + 1]
        assert D[yy, xx] == (s + 2) >> 2


@pytest.mark.parametrize("W,H,L,wl,hl,Lcap,Lf,wf,hf", [
    (320, 180, 0, 320, 180, 3, 0, 320, 90),
    (720, 576, 1, 360, 288, 5, 0, 720, 288),
    (1280, 720, 2, 320, 180, 5, 1, 640, 180),
    (1920, 1080, 2, 480, 270, 6, 1, 960, 270),
    (2048, 1080, 2, 512, 270, 6, 1, 1024, 270),
    (3840, 2160, 3, 480, 270, 7, 2, 960, 270),
])
def test_geometry_of_formats(orc, params, W, H, L, wl, hl, Lcap, Lf, wf, hf):
    g = orc.geometry(W, H, params)
    assert g["L"] == L and g["dims"][L] == (wl, hl)
    assert g["Lcap"] == Lcap and g["Lf"] == Lf and g["field"] == (wf, hf)


def test_geometry_2k_coarse_levels(orc, params):
    g = orc.geometry(2048, 1080, params)
    assert g["dims"][3:7] == [(256, 135), (128, 67), (64, 33), (32, 16)]


def test_too_small_rejected(orc, params):
    with pytest.raises(ValueError):
        orc.geometry(15, 100, params)
    with pytest.raises(ValueError):
        orc.geometry(100, 15, params)


def test_cosited_lower_field_on_vertical_ramp_lf0(orc, params):
    # 320x180: Lf = 0, fields are rows 2y (U) and 2y+1 (D).  On a vertical ramp
    # Y[r] = r the lower field halfway between rows 2y-1 and 2y+1 is row 2y,
    # i.e. the upper field itself (row 0 reads D[-1] as D[0]).
    Y = np.repeat(np.arange(180, dtype=np.uint8)[:, None], 320, axis=1)
    lv = orc.levels(Y, params)
    U, D, Dc = lv[("U", 0)], lv[("D", 0)], lv[("Dc", 0)]
    assert np.all(U[:, 0] == 2 * np.arange(90)) and np.all(D[:, 0] == 2 * np.arange(90) + 1)
    assert np.array_equal(Dc[1:], U[1:])
    assert np.array_equal(Dc[0], D[0])


def test_cosited_lower_field_on_vertical_ramp_lf1(orc, params):
    # 1280x720 10-bit: L = 2, Lf = 1.  U_1[y] averages rows 4y, 4y+2 (centre
    # 4y+1), D_1[y] rows 4y+1, 4y+3 (centre 4y+2); on Y[r] = r the lower field
    # moved up by one full-resolution row is again the upper field:
    # (3 (4y+2) + (4y-2) + 2) >> 2 = 4y+1.
    Y = np.repeat(np.arange(720, dtype=np.uint16)[:, None], 1280, axis=1)
    lv = orc.levels(Y, params, bits=10)
    U, D, Dc = lv[("U", 1)], lv[("D", 1)], lv[("Dc", 1)]
    y = np.arange(180)
    assert np.all(U[:, 5] == 4 * y + 1) and np.all(D[:, 5] == 4 * y + 2)
    assert np.array_equal(Dc[1:], U[1:])


def test_cosited_lower_field_weights(orc, params):
    # Row y of the resampled plane lies 1/p of a field row above D[y]
    # (p = 2^(Lf+1) full-resolution rows per field row), rounded half up;
    # checked at sampled points on random frames at Lf = 0, 1, 2.
    rng = np.random.default_rng(11)
    for W, H, bits, Lf in ((320, 180, 8, 0), (2048, 1080, 8, 1), (3840, 2160, 10, 2)):
        Y = rng.integers(0, (1 << bits), size=(H, W)).astype(np.uint8 if bits == 8 else np.uint16)
        lv = orc.levels(Y, params, bits=bits)
        D = lv[("D", Lf)].astype(np.int64)
        Dc = lv[("Dc", Lf)].astype(np.int64)
        p = 2 << Lf
        for (yy, xx) in [(0, 0), (1, 3), (50, 100), (D.shape[0] - 1, D.shape[1] - 1)]:
            prev = D[max(yy - 1, 0), xx]
            assert Dc[yy, xx] == ((p - 1) * D[yy, xx] + prev + p // 2) // p
