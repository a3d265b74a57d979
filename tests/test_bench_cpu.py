"""bench.py on the CPU: its command-line contract (one GPU only; every leg's
switch exists) and the algorithmic bytes per frame behind the pyramid
kernel's roofline, recomputed here from the level and field sizes."""
import math
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""          # no JSON line: nothing was measured


def test_every_leg_has_its_switch():
    r = subprocess.run([sys.executable, BENCH, "--help"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--streams", "--no-cpu-baseline", "--no-plain", "--no-clip",
                 "--clip-chunk", "--clip-only", "--no-mix", "--no-serve", "--no-stress", "--copy-only"):
        assert flag in r.stdout, flag


def _expected_k1_bytes(W, H, k_max, wmax=512):
    """Y read once; levels L .. min(L + ceil(log2(k_max + 1)), Lcap) and both
    fields at L - 1 written once; one 256-bin uint16 histogram per 64 x 16
    tile of level L."""
    sizes = []
    w, h = W, H
    while w > 0 and h > 0:
        sizes.append((w, h))
        w, h = w // 2, h // 2
    L = next(i for i, (w, _) in enumerate(sizes) if w <= wmax)
    Lcap = max(i for i, (w, h) in enumerate(sizes) if i >= L and w // 8 >= 2 and h // 8 >= 2)
    top = min(L + math.ceil(math.log2(k_max + 1)), Lcap)
    levels = sum(w * h for w, h in sizes[L:top + 1])
    Lf = max(0, L - 1)
    fields = 2 * (W >> Lf) * ((H // 2) >> Lf)
    wl, hl = sizes[L]
    tiles = math.ceil(wl / 64) * math.ceil(hl / 16)
    return W * H + levels + fields + tiles * 256 * 2


def test_pyramid_bytes_per_frame(orc, params):
    sys.path.insert(0, ROOT)
    import bench
    p = dict(params, k_max=8)
    g = orc.geometry(2048, 1080, p)
    got = bench.k1_bytes_per_frame(g, 2048, 1080, 8)
    assert got == _expected_k1_bytes(2048, 1080, 8) == 3018432
