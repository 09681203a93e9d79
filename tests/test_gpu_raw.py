"""pcr_resolve_raw: the framebuffer's words in one linear layout equal the
oracle's keys (closest point) and depth / sum words (HQ, Sec. 3.5), for the
two-word, robust and packed sum layouts."""
import numpy as np
import pytest

from gpu_util import oracle_frame, read_fb, render_frame, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu


def cloud(seed, n, W, H):
    """A dense cluster (tens of points per pixel, a few of them within the
    blend window; far below the packed form's 1023-point bound) plus points
    behind the camera and off-screen."""
    rng = np.random.default_rng(seed)
    m = synth.mvp((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, fovy=50.0)
    p = np.empty(n, synth.POINT_DTYPE)
    xyz = rng.uniform(-1.6, 1.6, (n, 3))
    xyz[: n // 10, 2] = rng.uniform(5.0, 9.0, n // 10)       # behind the eye
    xyz[n // 10: n // 5, 0] *= 8.0                            # mostly off-screen
    p["x"], p["y"], p["z"] = xyz.T
    p["rgba"] = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return p, m


@pytest.mark.parametrize("variant", [pcr.BASIC, pcr.DEDUP, pcr.HQ, pcr.HQ | pcr.F_HQ_ROBUST,
                                     pcr.HQ | pcr.F_HQ_PACKED, pcr.HQ | pcr.F_HQ_ROBUST | pcr.F_PLAIN])
@pytest.mark.parametrize("size", [(48, 32), (67, 29)])
def test_raw_words_equal_the_oracle(orc, variant, size):
    W, H = size
    pts, m = cloud(7, 30_011, W, H)
    efb, _ = oracle_frame(orc, pts, m, W, H, variant)
    fb, _ = render_frame(upload(pts), m, W, H, variant)
    raw = pcr.resolve_raw(fb, W, H, variant).cpu().numpy().view(np.uint64)
    npix = W * H
    if (variant & 0xFF) != pcr.HQ:
        assert raw.shape == (npix,)
        assert np.array_equal(raw, efb)
        return
    D, RG, BA = efb
    assert raw.shape == (3 * npix,)
    assert np.array_equal(raw[:npix], D.astype(np.uint64))
    assert np.array_equal(raw[npix:2 * npix], RG)
    assert np.array_equal(raw[2 * npix:], BA)
    assert (BA & 0xFFFFFFFF).max() >= 2                   # some pixel blends several points


def test_raw_two_word_is_the_stored_layout(orc):
    """For the two-word HQ layout the raw planes are the stored words, moved."""
    W, H = 40, 30
    pts, m = cloud(3, 12_000, W, H)
    fb, _ = render_frame(upload(pts), m, W, H, pcr.HQ)
    D, RG, BA = read_fb(fb, W, H, pcr.HQ)
    raw = pcr.resolve_raw(fb, W, H, pcr.HQ).cpu().numpy().view(np.uint64)
    assert np.array_equal(raw, np.concatenate([D.astype(np.uint64), RG, BA]))
