"""GPU parity of the dense inverse search flow pair measure (search = 2).

The device path evaluates the same sequential definition in IEEE double with
no contraction and every sum in the oracle's order, so the flow field and the
four measures must equal the oracle's bit for bit, on textured, translated,
sub-pixel, ramp, noise, flat and minimum-size planes, at the 2K working and
field-level shapes, in 8 and 10 bits; and the device-pointer entry (8-bit
planes with a row pitch, caller's scratch) must give what the host entry gives.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def fp(params):
    return dict(params, search=2)


def _texture(seed, size=256, hi=235):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.gen.texture(rng, size, 3.0, 16, hi).astype(np.uint16)


def _field(x, y):
    return 120 + 40 * np.sin(x / 7.0) * np.cos(y / 9.0) + 30 * np.sin((x + 2 * y) / 11.0)


def _cases():
    rng = np.random.default_rng(17)
    tex = _texture(11)
    out = []
    out.append(("identical", tex[:64, :96], tex[:64, :96].copy(), 8))
    for d in ((3, -2), (9, -4), (-6, 5)):
        out.append((f"shift{d}", tex[:96, :128], np.roll(tex, (d[1], d[0]), (0, 1))[:96, :128], 8))
    y, x = np.mgrid[0:96, 0:128].astype(np.float64)
    out.append(("subpixel", np.rint(_field(x, y)).astype(np.uint16),
                np.rint(_field(x - 1.5, y + 0.75)).astype(np.uint16), 8))
    y2, x2 = np.mgrid[0:48, 0:64]
    out.append(("ramp", (x2 + 2 * y2 + 40).astype(np.uint16), (x2 - 3 + 2 * (y2 + 2) + 40).astype(np.uint16), 8))
    out.append(("noise", rng.integers(0, 256, (40, 56)).astype(np.uint16),
                rng.integers(0, 256, (40, 56)).astype(np.uint16), 8))
    out.append(("flat", np.full((32, 40), 77, np.uint16), np.full((32, 40), 90, np.uint16), 8))
    for h, w in ((8, 8), (15, 9), (17, 33), (23, 50)):
        out.append((f"small{h}x{w}", rng.integers(0, 256, (h, w)).astype(np.uint16),
                    rng.integers(0, 256, (h, w)).astype(np.uint16), 8))
    t10 = _texture(5, hi=1000)
    out.append(("10bit", t10[:80, :112], np.roll(t10, (2, -3), (0, 1))[:80, :112], 10))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_flow_pair_bitwise(vsa, orc, params, case):
    name, I, J, bits = case
    print(f"flow pair {name} {I.shape} {bits}-bit", flush=True)
    ref = orc.flow_pair(I, J, fp(params))
    got = vsa.debug_flow_pair(I, J, fp(params), bit_depth=bits)
    assert np.array_equal(got["flow"].view(np.uint64), ref["flow"].view(np.uint64)), name
    for k in ("ncc", "swr", "amm", "act"):
        assert np.float64(got[k]).view(np.uint64) == np.float64(ref[k]).view(np.uint64), (name, k)
    assert got["static"] == ref["static"]


def _levels_2k(orc, params):
    spec = synth.make_c2(seed=2, T=1500, W=2048, H=1080, k_dis=8)
    fr = synth.render(spec, [100, 101])
    out = []
    for f in fr:
        lv = orc.levels(f, params)
        out.append(lv)
    return out


def test_flow_pair_2k_levels(vsa, orc, params):
    """Consecutive frames of the 2K clip at the working level (512 x 270) and
    their upper fields at the field level (1024 x 270)."""
    lv = _levels_2k(orc, params)
    g = orc.geometry(2048, 1080, params)
    for key in (("F", g["L"]), ("U", g["Lf"])):
        I, J = lv[0][key], lv[1][key]
        print(f"flow pair 2K {key} {I.shape}", flush=True)
        ref = orc.flow_pair(I, J, fp(params))
        got = vsa.debug_flow_pair(I, J, fp(params), bit_depth=8)
        assert np.array_equal(got["flow"].view(np.uint64), ref["flow"].view(np.uint64)), key
        for k in ("ncc", "swr", "amm", "act"):
            assert got[k] == ref[k], (key, k)


def test_flow_pair_device_entry(vsa, params):
    """8-bit device planes with a row pitch wider than the row, the caller's
    scratch, on a HIP stream: the host entry's results and flow."""
    import torch
    tex = _texture(23)
    I, J = tex[:90, :130], np.roll(tex, (4, -2), (0, 1))[:90, :130]
    ref = vsa.debug_flow_pair(I, J, fp(params), bit_depth=8)
    dI = torch.zeros((90, 160), dtype=torch.uint8, device="cuda:0")
    dJ = torch.zeros((90, 160), dtype=torch.uint8, device="cuda:0")
    dI[:, :130] = torch.from_numpy(I.astype(np.uint8)).to("cuda:0")
    dJ[:, :130] = torch.from_numpy(J.astype(np.uint8)).to("cuda:0")
    scratch = torch.empty(vsa.flow_scratch_bytes(130, 90), dtype=torch.uint8, device="cuda:0")
    res = torch.zeros(5, dtype=torch.float64, device="cuda:0")
    flow = torch.zeros((90, 130, 2), dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    vsa.flow_pair(dI[:, :130], dJ[:, :130], scratch, res, fp(params), flow=flow, stream=s.cuda_stream)
    s.synchronize()
    r = res.cpu().numpy()
    assert np.array_equal(flow.cpu().numpy().view(np.uint64), ref["flow"].view(np.uint64))
    assert [r[0], r[1], r[2], r[3]] == [ref["ncc"], ref["swr"], ref["amm"], ref["act"]]
    assert int(r[4]) == ref["static"]
    # a scratch buffer one byte short is refused
    with pytest.raises(vsa.VsaError):
        vsa.flow_pair(dI[:, :130], dJ[:, :130], scratch[:-1], res, fp(params))
