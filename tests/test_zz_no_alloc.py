"""pcr_render_chunks_static (the chunked frame without caller scratch, for
callers that cannot allocate) against pcr_render_chunks on the same chunk
tables, bit for bit, called through the C ABI: two calls in a row on every
variant, the second with a smaller table (fewer chunks and points), so that the
library's array still holds the first call's offsets when the second runs."""
import ctypes

import numpy as np
import pytest

from gpu_util import assert_same_fb, oracle_frame, read_fb, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu


def table_of(pts_dev, sizes):
    offs = np.concatenate([[0], np.cumsum(sizes)])
    base = pts_dev.data_ptr()
    return pcr.chunk_table([(base + 16 * int(offs[c]), int(sizes[c])) for c in range(len(sizes))])


def frame(L, table, nchunks, m, W, H, variant, static):
    """clear + chunked render + resolve through the C ABI; (fb, image)."""
    import torch
    fb = pcr.alloc_fb(W, H, variant)
    s = torch.cuda.current_stream().cuda_stream
    mv = (ctypes.c_float * 16)(*[float(x) for x in np.asarray(m, np.float32).reshape(16)])
    assert L.pcr_fb_clear(fb.data_ptr(), W, H, variant, s) == 0
    if static:
        rc = L.pcr_render_chunks_static(table.data_ptr(), nchunks, mv, W, H, variant, fb.data_ptr(), None, s)
    else:
        scratch = torch.empty(max(256, L.pcr_chunks_scratch_bytes(nchunks)), dtype=torch.uint8, device="cuda")
        rc = L.pcr_render_chunks(table.data_ptr(), nchunks, mv, W, H, variant, fb.data_ptr(), scratch.data_ptr(),
                                 scratch.numel(), None, s)
    assert rc == 0, L.pcr_last_error().decode()
    img = torch.empty(W * H, dtype=torch.int32, device="cuda")
    assert L.pcr_resolve(fb.data_ptr(), W, H, variant, img.data_ptr(), s) == 0
    torch.cuda.synchronize()
    return fb, img.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("variant", [pcr.BASIC, pcr.DEDUP, pcr.HQ])
def test_static_scratch_matches_caller_scratch(orc, variant):
    L = pcr.lib()
    rng = np.random.default_rng(21)
    W, H = 640, 360
    pts = synth.terrain(1_200_000, seed=2)
    pts = pts[orc.reorder(pts, 1, 128, 3)]
    d = upload(pts)
    m = synth.terrain_oblique(W, H)
    big = np.maximum(1, rng.lognormal(np.log(2400), 0.8, 400)).astype(np.int64)
    big = np.concatenate([[0, 1, 255, 256, 257], big])
    big = big[np.cumsum(big) <= len(pts)]
    small = big[:37]
    for k, sizes in enumerate((big, small)):         # second call: fewer chunks, fewer points
        tab = table_of(d, sizes)
        fb_s, img_s = frame(L, tab, len(sizes), m, W, H, variant, static=True)
        fb_r, img_r = frame(L, tab, len(sizes), m, W, H, variant, static=False)
        assert_same_fb(read_fb(fb_s, W, H, variant), read_fb(fb_r, W, H, variant), variant)
        assert np.array_equal(img_s, img_r), (variant, k)
        if k == 0:
            _, eimg = oracle_frame(orc, pts[: int(sizes.sum())], m, W, H, variant)
            assert np.array_equal(img_s, eimg)
        assert img_s.any()
