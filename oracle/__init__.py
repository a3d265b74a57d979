"""ctypes binding of the CPU oracle (``liborc.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  The
oracle is a plain scalar C++ implementation of the measure engine written from
the paper's definitions (Sec. III); it shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SRC = os.path.join(HERE, "orc.cpp")

F_HAS_PAIR, F_STATIC, F_FAST_FIRED, F_IN_TRANSITION = 1, 2, 4, 8
F_KEYFRAME, F_SHOT_START, F_ANALYZED = 16, 32, 64


def build(force: bool = False) -> str:
    """Compile liborc.so with g++ (plain -O2, no FP contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
        os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "orc.h"))
    ):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared",
             "-fPIC", "-Wall", "-Wextra", "-o", tmp, SRC]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [
        ("block", C.c_int32), ("radius", C.c_int32), ("wmax", C.c_int32),
        ("lf_offset", C.c_int32), ("k_max", C.c_int32), ("a_static_fx", C.c_int32),
        ("w_hist", C.c_int32), ("n_ss", C.c_int32),
        ("a0", C.c_double), ("rho_f", C.c_double), ("theta_f", C.c_double), ("theta_f0", C.c_double),
        ("rho_d", C.c_double), ("theta_d", C.c_double), ("gamma", C.c_double),
        ("tau_c", C.c_double), ("eps", C.c_double), ("tau_p", C.c_double),
        ("theta_kf", C.c_double), ("search", C.c_int32), ("refine", C.c_int32),
    ]


FRAME_DTYPE = np.dtype([
    ("frame", "<i8"), ("flags", "<i4"), ("shot_id", "<i4"), ("boundary", "<i4"),
    ("boundary_k", "<i4"), ("ncc", "<f8"), ("swr", "<f8"), ("amm", "<f8"), ("act", "<f8"),
    ("mom", "<i8", (5,)), ("n_pix", "<i8"), ("amm_num", "<i8"), ("n_blocks", "<i4"),
    ("field_mask", "<u4"), ("v", "<f8", (3,)), ("h_mean", "<f8"), ("h_std", "<f8"), ("h_mad", "<f8"),
])
SHOT_DTYPE = np.dtype([
    ("shot_id", "<i4"), ("pad0", "<i4"), ("first", "<i8"), ("last", "<i8"),
    ("in_boundary", "<i4"), ("in_k", "<i4"), ("sampling", "<i4"), ("pulldown_phase", "<i4"),
    ("n_analyzed", "<i4"), ("final", "<i4"),
])
KEY_DTYPE = np.dtype([("kind", "<i4"), ("ref", "<i4"), ("oth", "<i4"), ("ref_field", "<i4"),
                      ("oth_field", "<i4"), ("level", "<i4")])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_geometry.argtypes = [C.c_int32, C.c_int32, C.POINTER(Params), P, C.c_int32]
        L.orc_downscale.argtypes = [P, C.c_int32, C.c_int32, P]
        L.orc_levels.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.c_int32,
                                 C.POINTER(Params), P, C.c_int64, C.POINTER(C.c_int64)]
        L.orc_pair.argtypes = [P, P, C.c_int32, C.c_int32, C.POINTER(Params), C.c_int32,
                               P, P, P, P]
        L.orc_finish.argtypes = [P, C.c_double, P]
        L.orc_flow_pair.argtypes = [P, P, C.c_int32, C.c_int32, C.POINTER(Params), P, P, P]
        L.orc_intensity.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, P]
        L.orc_run_clip.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_int64,
                                   C.c_int32, C.c_int32, C.POINTER(Params), P, P, C.c_int32,
                                   C.POINTER(C.c_int32), P, C.c_int32, C.POINTER(C.c_int32), P]
        L.orc_decide_injected.argtypes = [C.c_int32, P, P, P, P, P, P, P, C.c_int32,
                                          C.POINTER(Params), P, P, C.c_int32,
                                          C.POINTER(C.c_int32), P, C.c_int32,
                                          C.POINTER(C.c_int32)]
        for f in ("orc_geometry", "orc_downscale", "orc_levels", "orc_pair", "orc_finish", "orc_flow_pair",
                  "orc_intensity", "orc_run_clip", "orc_decide_injected"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def make_params(d: dict) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        setattr(p, name, d[name])
    return p


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with status {rc}")


def geometry(W, H, params):
    out = np.zeros(128, np.int32)
    _check(lib().orc_geometry(W, H, make_params(params), _ptr(out), out.size), "orc_geometry")
    L, Lcap, Lf, nl = (int(x) for x in out[:4])
    dims = [(int(out[4 + 2 * l]), int(out[5 + 2 * l])) for l in range(nl)]
    wf, hf = int(out[4 + 2 * nl]), int(out[5 + 2 * nl])
    return {"L": L, "Lcap": Lcap, "Lf": Lf, "dims": dims, "field": (wf, hf)}


def downscale(plane):
    s = np.ascontiguousarray(plane, dtype=np.uint16)
    h, w = s.shape
    d = np.zeros((h // 2, w // 2), np.uint16)
    _check(lib().orc_downscale(_ptr(s), w, h, _ptr(d)), "orc_downscale")
    return d


def levels(Y, params, bits=8):
    """Frame levels L..Lcap, the two fields at Lf and the lower field on the
    upper field's rows ("Dc", what field pairs read), as a dict of uint16 planes."""
    Y = np.ascontiguousarray(Y)
    H, W = Y.shape
    g = geometry(W, H, params)
    n = C.c_int64(0)
    pitch = Y.strides[0]
    p = make_params(params)
    _check(lib().orc_levels(_ptr(Y), W, H, pitch, bits, p, None, 0, C.byref(n)), "orc_levels")
    out = np.zeros(n.value, np.uint16)
    _check(lib().orc_levels(_ptr(Y), W, H, pitch, bits, p, _ptr(out), out.size, C.byref(n)),
           "orc_levels")
    res, k = {}, 0
    for l in range(g["L"], g["Lcap"] + 1):
        w, h = g["dims"][l]
        res[("F", l)] = out[k:k + w * h].reshape(h, w)
        k += w * h
    wf, hf = g["field"]
    res[("U", g["Lf"])] = out[k:k + wf * hf].reshape(hf, wf)
    k += wf * hf
    res[("D", g["Lf"])] = out[k:k + wf * hf].reshape(hf, wf)
    k += wf * hf
    res[("Dc", g["Lf"])] = out[k:k + wf * hf].reshape(hf, wf)
    return res


def pair(I, J, params, force_zero_mv=False):
    I = np.ascontiguousarray(I, dtype=np.uint16)
    J = np.ascontiguousarray(J, dtype=np.uint16)
    h, w = I.shape
    B = (w // 8) * (h // 8)
    mv = np.zeros((max(B, 1), 2), np.int8)
    sad = np.zeros(max(B, 1), np.int32)
    ints = np.zeros(9, np.int64)
    dbl = np.zeros(4, np.float64)
    _check(lib().orc_pair(_ptr(I), _ptr(J), w, h, make_params(params), int(force_zero_mv),
                          _ptr(mv), _ptr(sad), _ptr(ints), _ptr(dbl)), "orc_pair")
    keys = ("sx", "sy", "sxx", "syy", "sxy", "n", "a", "B", "static")
    out = {k: int(v) for k, v in zip(keys, ints)}
    out.update(ncc=float(dbl[0]), swr=float(dbl[1]), amm=float(dbl[2]), act=float(dbl[3]))
    out["mv"] = mv[:B].reshape(h // 8, w // 8, 2)
    out["sad"] = sad[:B].reshape(h // 8, w // 8)
    return out


def flow_pair(I, J, params):
    """Pair measure with the dense inverse search flow (search = 2):
    {"flow": [h, w, 2] (dx, dy), "ncc", "swr", "amm", "act", "static"}."""
    I = np.ascontiguousarray(I, dtype=np.uint16)
    J = np.ascontiguousarray(J, dtype=np.uint16)
    h, w = I.shape
    flow = np.zeros((h, w, 2), np.float64)
    dbl = np.zeros(4, np.float64)
    st = C.c_int32(0)
    _check(lib().orc_flow_pair(_ptr(I), _ptr(J), w, h, make_params(params), _ptr(flow), _ptr(dbl), C.byref(st)),
           "orc_flow_pair")
    return {"flow": flow, "ncc": float(dbl[0]), "swr": float(dbl[1]), "amm": float(dbl[2]), "act": float(dbl[3]),
            "static": int(st.value)}


def intensity(plane, bits=8):
    """Sec. III.A unary measure of one plane: (histogram int64[2^bits],
    {"n", "s1", "s2", "m"}, (mean, std, mad))."""
    q = np.ascontiguousarray(plane, dtype=np.uint16)
    h, w = q.shape
    hist = np.zeros(1 << bits, np.int64)
    ints = np.zeros(4, np.int64)
    out = np.zeros(3, np.float64)
    _check(lib().orc_intensity(_ptr(q), w, h, bits, _ptr(hist), _ptr(ints), _ptr(out)), "orc_intensity")
    return hist, dict(zip(("n", "s1", "s2", "m"), (int(v) for v in ints))), tuple(float(v) for v in out)


def finish(ints8, a0):
    v = np.ascontiguousarray(ints8, dtype=np.int64)
    out = np.zeros(4, np.float64)
    _check(lib().orc_finish(_ptr(v), float(a0), _ptr(out)), "orc_finish")
    return out


def run_clip(frames, params, bits=8, dense=False, want_mv=False):
    """Offline sequential pass over frames[T, H, W] (uint8 or uint16)."""
    frames = np.ascontiguousarray(frames)
    T, H, W = frames.shape
    g = geometry(W, H, params)
    wl, hl = g["dims"][g["L"]]
    B = (wl // 8) * (hl // 8)
    recs = np.zeros(T, FRAME_DTYPE)
    shots = np.zeros(T + 1, SHOT_DTYPE)
    kcap = T * (4 + 2 * (params["k_max"] + 2)) + 16
    keys = np.zeros(kcap, KEY_DTYPE)
    ns, nk = C.c_int32(0), C.c_int32(0)
    mv = np.zeros((max(T - 1, 1), B, 2), np.int8) if want_mv else None
    _check(lib().orc_run_clip(_ptr(frames), T, W, H, frames.strides[1], frames.strides[0], bits,
                              int(dense), make_params(params), _ptr(recs), _ptr(shots),
                              shots.size, C.byref(ns), _ptr(keys), kcap, C.byref(nk), _ptr(mv)),
           "orc_run_clip")
    out = {"frames": recs, "shots": shots[:ns.value].copy(), "keys": keys[:nk.value].copy()}
    if want_mv:
        out["mv"] = mv[:T - 1].reshape(T - 1, hl // 8, wl // 8, 2)
    return out


def decide_injected(seq, params, dense=False):
    """Sequential pass over injected measure sequences (see orc.h)."""
    T = len(seq["act"])
    kw = params["k_max"] + 2
    act = np.ascontiguousarray(seq["act"], np.float64)
    swr = np.ascontiguousarray(seq["swr"], np.float64)
    stat = np.ascontiguousarray(seq["static"], np.uint8)
    v = np.ascontiguousarray(seq["v"], np.float64).reshape(T, 3)
    F = np.ascontiguousarray(seq["F"], np.float64).reshape(T, kw)
    S = np.ascontiguousarray(seq["S"], np.float64).reshape(T, kw)
    P = np.ascontiguousarray(seq["P"], np.float64).reshape(T, kw)
    recs = np.zeros(T, FRAME_DTYPE)
    shots = np.zeros(T + 1, SHOT_DTYPE)
    kcap = T * (4 + 2 * kw) + 16
    keys = np.zeros(kcap, KEY_DTYPE)
    ns, nk = C.c_int32(0), C.c_int32(0)
    _check(lib().orc_decide_injected(T, _ptr(act), _ptr(swr), _ptr(stat), _ptr(v), _ptr(F),
                                     _ptr(S), _ptr(P), int(dense), make_params(params),
                                     _ptr(recs), _ptr(shots), shots.size, C.byref(ns),
                                     _ptr(keys), kcap, C.byref(nk)), "orc_decide_injected")
    return {"frames": recs, "shots": shots[:ns.value].copy(), "keys": keys[:nk.value].copy()}
