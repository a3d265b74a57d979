"""Engine configuration on the GPU: parameters given as JSON, and the launch
tuner's cache file."""
import json

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_params_json_engine(vsa, params):
    """An engine configured from the JSON text gives the records and shots of
    one configured from the parameter struct."""
    frames = synth.render(synth.make_c1(T=40))
    p = dict(params, k_max=6, theta_kf=2.5)
    a = vsa.run_clip(frames, p)
    b = vsa.run_clip(frames, None, params_json=json.dumps(p))
    for name in a["frames"].dtype.names:
        x, y = a["frames"][name], b["frames"][name]
        if x.dtype.kind == "f":
            assert np.array_equal(x.view(np.uint64), y.view(np.uint64)), name
        else:
            assert np.array_equal(x, y), name
    assert np.array_equal(a["shots"], b["shots"])
    with pytest.raises(vsa.VsaError):
        vsa.Engine(max_streams=1, params_json='{"k_max": "eight"}')


def _run_steps(vsa, e, frames, n_streams, steps):
    import torch
    dev = torch.from_numpy(frames).to("cuda:0")
    T, H, W = frames.shape
    sids = np.array([e.stream_open(W, H, 8) for _ in range(n_streams)], np.int32)
    plane = H * W
    pitches = np.full(n_streams, W, np.int64)
    for s in range(steps):
        ptrs = np.array([dev.data_ptr() + ((s + 5 * i) % T) * plane for i in range(n_streams)], np.uint64)
        assert e.stream_push_batch(sids, ptrs, pitches, vsa.SRC_DEVICE_BORROW, None) == 0
        e.step()
    e.sync()


def test_autotune_cache(vsa, params, tmp_path):
    """A tuned bucket is written to the cache file; a new engine reading the
    file takes that choice for the bucket without timing any window."""
    path = tmp_path / "tune.txt"
    frames = synth.render(synth.make_c1(T=64))
    with vsa.Engine(max_streams=8, params=params, autotune_cache=str(path)) as e:
        _run_steps(vsa, e, frames, 8, 260)
        tuned = {b: t["best"] for b, t in e.tuning().items() if t["best"] >= 0}
    assert tuned, "no bucket settled"
    lines = path.read_text().splitlines()
    assert len(lines) >= len(tuned)
    with vsa.Engine(max_streams=8, params=params, autotune_cache=str(path)) as e2:
        t2 = e2.tuning()
        for b, best in tuned.items():
            assert t2[b]["best"] == best
            assert all(c["windows"] == 0 for c in t2[b]["candidates"])
        _run_steps(vsa, e2, frames, 8, 100)
        t3 = e2.tuning()
        for b in tuned:
            assert all(c["windows"] == 0 for c in t3[b]["candidates"])
    # a cache file of another search mode or CU count is not used
    other = tmp_path / "other.txt"
    other.write_text("\n".join(l.replace("search 0", "search 1") for l in lines) + "\n")
    with vsa.Engine(max_streams=8, params=params, autotune_cache=str(other)) as e3:
        assert all(t["best"] < 0 for t in e3.tuning().values())
