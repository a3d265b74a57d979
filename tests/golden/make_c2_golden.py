"""Writes c2_seed2_k8.npz: the oracle's records for the whole 1500-frame
2048x1080 clip of the 2K workload (seed 2, 8-frame dissolves), k_max 8,
sparse schedule, with the default parameters.

The expected values come from the oracle alone (oracle/); the frames come
from the seeded generator (synth/).  Each frame's 64-bit BLAKE2b digest is
stored beside the records, so a test can check that it renders the same
frames before it compares anything.

    python tests/golden/make_c2_golden.py [--workers N]

takes about three minutes on eight cores (the oracle is single-threaded).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "c2_seed2_k8.npz")
SEED, T, W, H, K_MAX = 2, 1500, 2048, 1080, 8


def spec():
    import synth
    return synth.make_c2(seed=SEED, T=T, W=W, H=H, k_dis=8)


def frame_digest(plane: np.ndarray) -> int:
    return int.from_bytes(hashlib.blake2b(np.ascontiguousarray(plane).tobytes(), digest_size=8).digest(), "little")


def _render(args):
    lo, hi = args
    import synth
    r = synth.Renderer(spec())
    return lo, np.stack([r.frame(t) for t in range(lo, hi)])


def render_all(workers: int) -> np.ndarray:
    out = np.empty((T, H, W), np.uint8)
    cuts = np.linspace(0, T, 4 * workers + 1).astype(int)
    with mp.get_context("spawn").Pool(workers) as pool:
        for lo, block in pool.imap_unordered(_render, list(zip(cuts[:-1], cuts[1:]))):
            out[lo:lo + len(block)] = block
        pool.close()
        pool.join()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    import oracle
    oracle.build()
    params = json.load(open(os.path.join(ROOT, "paper_2502_09202_amd", "params", "default.json")))
    params["k_max"] = K_MAX
    t0 = time.time()
    frames = render_all(args.workers)
    digests = np.array([frame_digest(f) for f in frames], np.uint64)
    t1 = time.time()
    ref = oracle.run_clip(frames, params)
    t2 = time.time()
    np.savez_compressed(OUT, frames=ref["frames"], shots=ref["shots"], keys=ref["keys"], digests=digests,
                        meta=np.array([SEED, T, W, H, K_MAX], np.int64))
    print(f"rendered in {t1 - t0:.0f} s, oracle {t2 - t1:.0f} s; {len(ref['shots'])} shots, "
          f"{len(ref['keys'])} sparse measures -> {OUT} ({os.path.getsize(OUT)} bytes)")


if __name__ == "__main__":
    main()
