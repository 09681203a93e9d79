"""GPU parity of the depth output of the resolve (linear w, window depth and
reverse-z) against the CPU oracle, bit for bit, on rendered frames and on
hand-built framebuffers that reach the reciprocal's slow range."""
import numpy as np
import pytest

from gpu_util import hq_depth_bytes, oracle_frame, render_frame, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu

MODES = [(pcr.DEPTH_LINEAR, 0.0, 0.0)] + [
    (pcr.DEPTH_HYPERBOLIC, *pcr.depth_coeffs(n, f, rev)) for n, f in ((0.1, 5000.0), (2.0, 3000.0))
    for rev in (False, True)] + [(pcr.DEPTH_HYPERBOLIC, 0.75, -3.0e-3)]


def bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def oracle_depth(orc, efb, W, H, variant, mode, a, b, empty):
    if (variant & 0xFF) == pcr.HQ:
        return orc.resolve_depth_hq(efb[0], W, H, mode, a, b, empty)
    return orc.resolve_depth_basic(efb, W, H, mode, a, b, empty)


def gpu_depth(fb, W, H, variant, mode, a, b, empty, with_rgba):
    import torch
    rgba = torch.empty(W * H, dtype=torch.int32, device="cuda") if with_rgba else None
    d, rgba = pcr.resolve_depth(fb, W, H, variant, mode, a, b, empty, rgba=rgba)
    torch.cuda.synchronize()
    return d.cpu().numpy(), (rgba.cpu().numpy().view(np.uint32) if with_rgba else None)


@pytest.mark.parametrize("variant", [pcr.BASIC, pcr.DEDUP, pcr.HQ])
@pytest.mark.parametrize("scene", ["terrain_2m_1080p", "sphere_1m_333x1", "dense_1x1"])
def test_depth_of_rendered_frames(orc, variant, scene):
    if scene == "terrain_2m_1080p":
        pts, m, W, H = synth.terrain(2_000_000, seed=2), synth.terrain_oblique(1920, 1080), 1920, 1080
    elif scene == "sphere_1m_333x1":
        pts, m, W, H = synth.sphere(1_000_000, seed=1), synth.sphere_view(333, 1), 333, 1
    else:
        pts, m, W, H = synth.sphere(50_000, seed=3), synth.sphere_view(1, 1), 1, 1
    efb, eimg = oracle_frame(orc, pts, m, W, H, variant)
    fb, img = render_frame(upload(pts), m, W, H, variant)
    assert np.array_equal(img, eimg)
    for k, (mode, a, b) in enumerate(MODES):
        want = oracle_depth(orc, efb, W, H, variant, mode, a, b, -7.5)
        got, rgba = gpu_depth(fb, W, H, variant, mode, a, b, -7.5, with_rgba=(k % 2 == 0))
        bad = np.nonzero(bits(got) != bits(want))[0]
        assert len(bad) == 0, (mode, a, b, len(bad), got[bad[:4]], want[bad[:4]])
        if rgba is not None:
            assert np.array_equal(rgba, eimg)


def extreme_depths():
    """Depth bits over the whole positive range: denormals, the ranges where
    the fast reciprocal needs the full division, 1.0, the largest float, inf."""
    rng = np.random.default_rng(8)
    special = np.array([1, 2, 0x007FFFFF, 0x00800000, 0x01000000, 0x013FFFFF, 0x3F800000, 0x7E800000,
                        0x7E800001, 0x7F000000, 0x7F7FFFFF, 0x7F800000], np.uint32)
    rand = rng.integers(1, 0x7F800001, 20_000, dtype=np.uint64).astype(np.uint32)
    return np.concatenate([special, rand])


@pytest.mark.parametrize("variant", [pcr.BASIC, pcr.HQ])
def test_depth_of_built_framebuffers(orc, variant):
    """Framebuffers written on the host (any stored depth is a valid input):
    every mode matches the oracle bit for bit, uncovered pixels included."""
    import torch
    dbits = extreme_depths()
    n = len(dbits) + 37                     # a ragged tail of uncovered pixels
    W, H = n, 1
    rng = np.random.default_rng(9)
    if variant == pcr.BASIC:
        keys = np.full(n, np.uint64(0xFFFFFFFFFFFFFFFF))
        keys[: len(dbits)] = (dbits.astype(np.uint64) << np.uint64(32)) | rng.integers(
            0, 2**32, len(dbits), dtype=np.uint64)
        perm = rng.permutation(n)
        keys = keys[perm]
        raw = keys.view(np.uint8)
        efb = keys
    else:
        D = np.full(n, 0xFFFFFFFF, np.uint32)
        D[: len(dbits)] = dbits
        D = D[rng.permutation(n)]
        S = np.zeros(2 * n, np.uint64)
        cov = D != 0xFFFFFFFF
        S[0::2][cov] = (np.uint64(200) << np.uint64(32)) | np.uint64(100)
        S[1::2][cov] = (np.uint64(50) << np.uint64(32)) | np.uint64(2)
        raw = np.zeros(hq_depth_bytes(W, H) + 16 * n, np.uint8)
        raw[: 4 * n] = D.view(np.uint8)
        raw[hq_depth_bytes(W, H):] = S.view(np.uint8)
        efb = (D, S[0::2], S[1::2])
    nb = pcr.fb_bytes(W, H, variant)
    assert len(raw) == nb
    fb = torch.from_numpy(np.concatenate([raw, np.zeros((-nb) % 8, np.uint8)]).view(np.int64)).to("cuda")
    for k, (mode, a, b) in enumerate(MODES):
        want = oracle_depth(orc, efb, W, H, variant, mode, a, b, float("inf"))
        got, rgba = gpu_depth(fb, W, H, variant, mode, a, b, float("inf"), with_rgba=(k % 2 == 1))
        bad = np.nonzero(bits(got) != bits(want))[0]
        assert len(bad) == 0, (mode, a, b, len(bad), got[bad[:4]], want[bad[:4]])
        if rgba is not None:
            exp = (orc.resolve_hq(efb[1], efb[2], W, H) if variant == pcr.HQ
                   else orc.resolve_basic(efb, W, H))
            assert np.array_equal(rgba, exp)


def test_depth_of_an_empty_frame():
    import torch
    W, H = 640, 360
    for variant in (pcr.BASIC, pcr.HQ):
        fb = pcr.alloc_fb(W, H, variant)
        pcr.fb_clear(fb, W, H, variant)
        d, _ = pcr.resolve_depth(fb, W, H, variant, pcr.DEPTH_HYPERBOLIC, 0.5, -0.25, 1.0)
        torch.cuda.synchronize()
        assert torch.all(d == 1.0)
