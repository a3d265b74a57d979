"""vsa_pair_noalloc (the pair measure with nothing allocated: every
intermediate in the library's fixed device array) against vsa_debug_pair,
the entry point it is a variant of (GPU).

Two calls in a row on the same array, the second with a smaller plane, each
equal to vsa_debug_pair on the same planes: motion field and integers
bit-exact, the doubles bitwise (the stated bar is 1e-6 on NCC).  Planes are
handed over in device memory, the first at the array's maximum size
(1024 x 1024) with a row pitch larger than the row, both sample widths.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _plane(rng, h, w, maxv):
    y, x = np.mgrid[0:h, 0:w]
    base = (np.sin(x / 5.0 + rng.uniform(0, 6)) + np.cos(y / 7.0 + rng.uniform(0, 6))) * 0.25 + 0.5
    return np.clip(np.rint(base * maxv) + rng.integers(-3, 4, size=(h, w)), 0, maxv).astype(np.uint16)


def _shift(I, dx, dy, rng, maxv):
    J = np.roll(np.roll(I.astype(np.int64), dy, axis=0), dx, axis=1) + rng.integers(-2, 3, size=I.shape)
    return np.clip(J, 0, maxv).astype(np.uint16)


def _noalloc(vsa, params, I, J, bits, pad):
    import torch
    lib = vsa.lib()
    h, w = I.shape
    dt = torch.uint8 if bits == 8 else torch.int16
    npdt = np.uint8 if bits == 8 else np.int16
    dev = "cuda:0"
    # planes inside wider buffers: row pitch = (w + pad) samples
    bI = torch.zeros((h, w + pad), dtype=dt, device=dev)
    bJ = torch.zeros((h, w + pad), dtype=dt, device=dev)
    bI[:, :w] = torch.from_numpy(I.astype(npdt)).to(dev)
    bJ[:, :w] = torch.from_numpy(J.astype(npdt)).to(dev)
    B = (w // 8) * (h // 8)
    mv = torch.zeros((B, 2), dtype=torch.int8, device=dev)
    ints = torch.zeros(9, dtype=torch.int64, device=dev)
    dbl = torch.zeros(4, dtype=torch.float64, device=dev)
    p = vsa.make_params(params)
    s = torch.cuda.current_stream()
    rc = lib.vsa_pair_noalloc(C.byref(p), bI.data_ptr(), bJ.data_ptr(), w, h, bI.stride(0) * bI.element_size(),
                              bits, 0, mv.data_ptr(), ints.data_ptr(), dbl.data_ptr(), s.cuda_stream)
    assert rc == 0, vsa.last_error()
    torch.cuda.synchronize()
    return mv.cpu().numpy().reshape(h // 8, w // 8, 2), ints.cpu().numpy(), dbl.cpu().numpy()


def _check(vsa, params, I, J, bits, pad, what):
    mv, ints, dbl = _noalloc(vsa, params, I, J, bits, pad)
    ref = vsa.debug_pair(I, J, params, bit_depth=bits)
    assert np.array_equal(mv, ref["mv"]), f"{what}: motion field"
    keys = ("sx", "sy", "sxx", "syy", "sxy", "n", "a", "B", "static")
    assert [int(v) for v in ints] == [ref[k] for k in keys], f"{what}: integers"
    assert abs(dbl[0] - ref["ncc"]) <= 1e-6, f"{what}: NCC"
    got = np.array(dbl, np.float64)
    want = np.array([ref["ncc"], ref["swr"], ref["amm"], ref["act"]], np.float64)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), f"{what}: doubles"


@pytest.mark.parametrize("bits", [8, 10])
def test_two_calls_second_smaller(vsa, params, bits):
    rng = np.random.default_rng(71 + bits)
    maxv = (1 << bits) - 1
    print(f"no-alloc pair, {bits}-bit: 1024x1024 then 136x80", flush=True)
    I = _plane(rng, 1024, 1024, maxv)
    _check(vsa, params, I, _shift(I, 5, -3, rng, maxv), bits, 64, "1024x1024")
    I = _plane(rng, 80, 136, maxv)
    _check(vsa, params, I, _shift(I, -7, 6, rng, maxv), bits, 3, "136x80")


def test_limits(vsa, params):
    """Sizes beyond the array's maximum, and bad pitches, fail with
    VSA_E_INVAL before anything is enqueued."""
    import torch
    lib = vsa.lib()
    p = vsa.make_params(params)
    buf = torch.zeros(2 * 1025 * 1025, dtype=torch.uint8, device="cuda:0")
    ptr = buf.data_ptr()
    assert lib.vsa_pair_noalloc(C.byref(p), ptr, ptr, 1025, 16, 1025, 8, 0, None, None, None, None) == vsa.E_INVAL
    assert lib.vsa_pair_noalloc(C.byref(p), ptr, ptr, 16, 1025, 16, 8, 0, None, None, None, None) == vsa.E_INVAL
    assert lib.vsa_pair_noalloc(C.byref(p), ptr, ptr, 64, 64, 63, 8, 0, None, None, None, None) == vsa.E_INVAL
    assert lib.vsa_pair_noalloc(C.byref(p), ptr + 1, ptr, 64, 64, 128, 10, 0, None, None, None, None) == vsa.E_INVAL
