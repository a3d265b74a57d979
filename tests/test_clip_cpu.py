"""Host arithmetic of the offline clip form (CPU): how vsa_clip_run splits a
clip into chunks.  The chunks must tile the clip exactly, in order, none
larger than the chunk size (the ring holds two chunks plus the deep check's
reach), the first one min(chunk, max(16, chunk / 4)) frames long so that the
decisions start early, every other one but the last a full chunk."""
import numpy as np
import pytest

CLIP_LENGTHS = [1, 2, 3, 15, 16, 17, 63, 64, 65, 255, 256, 257, 1500, 5000]


@pytest.mark.parametrize("C", [1, 2, 7, 16, 24, 64, 256, 512, 4096])
def test_chunks_tile_the_clip(vsa, C):
    for T in CLIP_LENGTHS:
        starts, counts = vsa.debug_clip_chunks(C, T)
        assert starts[0] == 0
        assert counts[0] == min(T, C, max(16, C // 4))
        assert np.all(counts >= 1) and np.all(counts <= C)
        assert np.array_equal(starts[1:], starts[:-1] + counts[:-1])
        assert starts[-1] + counts[-1] == T
        assert np.all(counts[1:-1] == C)


def test_chunk_arguments(vsa):
    assert vsa.debug_clip_chunks(0, 600)[0].tolist() == vsa.debug_clip_chunks(256, 600)[0].tolist()   # 0 = 256
    assert len(vsa.debug_clip_chunks(64, 0)[0]) == 0
    lib = vsa.lib()
    for chunk, T in ((-1, 10), (4097, 10), (16, -1)):
        assert lib.vsa_debug_clip_chunks(chunk, T, None, None, 0) == vsa.E_INVAL
