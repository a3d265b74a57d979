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


def test_pyramid_bytes_per_frame(params):
    sys.path.insert(0, ROOT)
    import bench
    p = dict(params, k_max=8)
    g = bench.geometry(2048, 1080, p)
    got = bench.k1_bytes_per_frame(g, 2048, 1080, 8)
    assert got == _expected_k1_bytes(2048, 1080, 8) == 3018432


def test_bench_geometry_matches_the_level_rule(orc, params):
    """bench.py sizes its bytes with its own geometry (not the oracle's); the
    two agree on every format of the workloads and some odd sizes."""
    sys.path.insert(0, ROOT)
    import bench
    for W, H in ((320, 180), (720, 576), (1280, 720), (1920, 1080), (2048, 1080), (3840, 2160), (4099, 2051),
                 (64, 32), (1001, 77)):
        a, b = bench.geometry(W, H, params), orc.geometry(W, H, params)
        assert (a["L"], a["Lf"], a["Lcap"], a["field"]) == (b["L"], b["Lf"], b["Lcap"], b["field"]), (W, H)
        assert a["dims"][:b["Lcap"] + 1] == b["dims"][:b["Lcap"] + 1], (W, H)


def test_trace_summary_between_markers(tmp_path):
    """The kernel-trace summary takes only the dispatches between the two
    marker kernels (the headline's timed steps)."""
    rows = ["Kind,Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp",
            "K,1,vsa::k_me<unsigned char>,0,500000",
            "K,2,at::cuda::spin_kernel(long),600000,601000",
            "K,3,vsa::k_me<unsigned char>,700000,710000",
            "K,4,vsa::k_me<unsigned char>,710000,730000",
            "K,5,\"vsa::k_pyramid<unsigned char, 2>\",710000,711000",
            "K,6,at::cuda::spin_kernel(long),800000,801000",
            "K,7,vsa::k_me<unsigned char>,900000,990000"]
    f = tmp_path / "kernel_trace.csv"
    f.write_text("\n".join(rows) + "\n")
    r = subprocess.run([sys.executable, BENCH, "--summarize-trace", str(f)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    line = next(l for l in r.stdout.splitlines() if "k_me" in l)
    assert line.split()[-5:] == ["2", "0.030", "15.00", "10.00", "20.00"]


def test_short_kernel_names():
    """Trace summaries name kernels without return type, namespaces and
    parameters, template arguments kept (so the phases of one template stay
    apart)."""
    sys.path.insert(0, os.path.dirname(BENCH))
    import bench
    assert bench.short_kernel_name(
        "void vsa::(anonymous namespace)::k_flow_list<2>(vsa::StreamDesc const*, int)") == "k_flow_list<2>"
    assert bench.short_kernel_name("void vsa::k_pyramid<unsigned char, 2>(vsa::StreamDesc const*)") == \
        "k_pyramid<unsigned char, 2>"
    assert bench.short_kernel_name("vsa::k_copy16(HIP_vector_type<unsigned int, 4u>*, long)") == "k_copy16"
    assert bench.short_kernel_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"
