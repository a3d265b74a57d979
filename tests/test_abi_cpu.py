"""The C-ABI library on the CPU: it loads, exports every symbol include/vsa.h
declares, its built-in defaults equal the shipped parameter file, and calls
fail cleanly (status codes, no crash) where no GPU is present."""
import ctypes as C
import json
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "vsa.h")).read()
    decl = re.findall(r"^(?:const\s+)?[A-Za-z_0-9]+\s*\*?\s*(vsa_[a-z_0-9]+)\(", text, re.M)
    return sorted(set(decl))


def test_header_declares_binding_symbols(vsa):
    assert declared_symbols() == sorted(vsa.SYMBOLS)


def test_library_exports_every_symbol(vsa):
    lib = vsa.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", vsa.LIB_PATH], capture_output=True, text=True).stdout
    for name in declared_symbols():
        assert re.search(rf"\bT {name}\b", out), name


def test_abi_version(vsa):
    assert vsa.abi_version() == 3


def test_defaults_match_parameter_file(vsa, params):
    d = vsa.default_params()
    assert set(d) == set(params)
    for k, v in params.items():
        assert d[k] == v, k


def test_errors_without_device(vsa):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(vsa.VsaError) as ei:
        vsa.Engine()
    assert ei.value.code in (vsa.E_DEVICE, vsa.E_INVAL)
    assert vsa.last_error()


def test_null_arguments(vsa):
    lib = vsa.lib()
    assert lib.vsa_engine_create(None, None) == vsa.E_INVAL
    lib.vsa_engine_destroy(None)   # no-op
    assert lib.vsa_step(None, None) == vsa.E_INVAL
    assert lib.vsa_sync(None) == vsa.E_INVAL
    assert lib.vsa_poll_frames(None, 0, None, 0) == vsa.E_INVAL
    assert lib.vsa_stream_footprint(None, None) == 0
    assert lib.vsa_debug_finish(None, 1, C.c_double(1.0), None) == vsa.E_INVAL


def test_engine_config_checks(vsa):
    # checked before any device call, so they run without a GPU
    with pytest.raises(vsa.VsaError) as ei:
        vsa.Engine(use_graph=1)
    assert ei.value.code == vsa.E_UNSUPPORTED and "graph" in vsa.last_error()
    for bad in (-1, 9):
        with pytest.raises(vsa.VsaError) as ei:
            vsa.Engine(me_wgs_per_cu=bad)
        assert ei.value.code == vsa.E_INVAL
    lib = vsa.lib()
    assert lib.vsa_collect(None, None) == vsa.E_INVAL
    assert lib.vsa_poll_frames_all(None, None, None, 0) == vsa.E_INVAL


def test_clip_config_checks(vsa):
    # checked before any device call, so they run without a GPU
    for kw in (dict(chunk=-1), dict(chunk=4097), dict(bit_depth=9), dict(k_max=16), dict(me_wgs_per_cu=9)):
        with pytest.raises(vsa.VsaError) as ei:
            vsa.Clip(64, 32, **kw)
        assert ei.value.code == vsa.E_INVAL, kw
    for w, h in ((15, 16), (16, 15), (0, 16)):
        with pytest.raises(vsa.VsaError) as ei:
            vsa.Clip(w, h)
        assert ei.value.code == vsa.E_INVAL
    lib = vsa.lib()
    assert lib.vsa_clip_create(None, None) == vsa.E_INVAL
    lib.vsa_clip_destroy(None)   # no-op
    assert lib.vsa_clip_run(None, None, 0, 0, 0, 0, None, None, 0, None) == vsa.E_INVAL
    assert lib.vsa_clip_counters(None, None, 0) == vsa.E_INVAL


def test_clip_without_device(vsa):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(vsa.VsaError) as ei:
        vsa.Clip(64, 32)
    assert ei.value.code == vsa.E_DEVICE
    assert vsa.last_error()


def test_params_from_json(vsa, params):
    """The library reads the package's parameter file as its own defaults,
    a partial object over the defaults, and refuses malformed objects."""
    import json
    import os
    here = os.path.join(os.path.dirname(vsa.__file__), "params", "default.json")
    got = vsa.params_from_json(open(here).read())
    ref = vsa.params_from_json("{}")
    assert got == ref
    assert got == {k: params[k] for k in got}
    part = vsa.params_from_json('{"k_max": 8, "theta_kf": 2.5e0, "search": 1}')
    assert part["k_max"] == 8 and part["theta_kf"] == 2.5 and part["search"] == 1
    assert {k: v for k, v in part.items() if k not in ("k_max", "theta_kf", "search")} == \
        {k: v for k, v in ref.items() if k not in ("k_max", "theta_kf", "search")}
    assert vsa.params_from_json(json.dumps({"rho_f": 2})) ["rho_f"] == 2.0
    for bad in ('{"k_max": 8.5}', '{"nope": 1}', '{"k_max" 8}', '{"k_max": 8,}', '[1]', '{"k_max": 8} x',
                '{"k_max": 3000000000}', '{"a0": }', '', '{"k_max": nan}', '{"a0": inf}', '{"a0": 0x10}',
                '{"k_max": -infinity}'):
        with pytest.raises(vsa.VsaError):
            vsa.params_from_json(bad)


def test_flow_scratch_sizes(vsa):
    """The flow pair's scratch size is host arithmetic: monotone in the plane,
    refused below one patch and at 2^31 samples or more (the kernels address
    a plane with 32-bit offsets)."""
    a = vsa.flow_scratch_bytes(512, 270)
    assert a > 0 and a % 256 == 0
    assert vsa.flow_scratch_bytes(1024, 270) > a > vsa.flow_scratch_bytes(256, 135)
    assert vsa.flow_scratch_bytes(8, 8) > 0
    for w, h in ((7, 8), (8, 7), (1 << 16, 1 << 15), (1 << 24, 8)):
        with pytest.raises(vsa.VsaError):
            vsa.flow_scratch_bytes(w, h)
    assert vsa.flow_scratch_bytes((1 << 16) - 1, 1 << 15) > 0
