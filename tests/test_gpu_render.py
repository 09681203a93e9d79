"""GPU parity of clear + render + resolve against the CPU oracle: bit-exact
framebuffers and images for every variant, flag set and launch shape."""
import numpy as np
import pytest

from gpu_util import assert_same_fb, oracle_frame, read_fb, render_frame, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu

B, D, HQ = pcr.BASIC, pcr.DEDUP, pcr.HQ
EZ, RD, LDS = pcr.F_EARLYZ, pcr.F_REDUCE, pcr.F_LDS
WV, PR = pcr.F_REDUCE_WAVE, pcr.F_REDUCE_PAIR
BASIC_FORMS = [B, B | EZ, B | RD, B | EZ | RD, B | WV, B | PR, B | EZ | WV, B | EZ | PR, B | LDS, B | LDS | EZ,
               B | LDS | RD, B | LDS | WV, B | LDS | EZ | RD, D, D | pcr.F_PLAIN, B | pcr.F_PLAIN]
HQ_FORMS = [HQ, HQ | EZ, HQ | RD, HQ | RD | EZ, HQ | WV, HQ | PR | EZ, HQ | LDS, HQ | LDS | EZ, HQ | LDS | RD,
            HQ | LDS | WV, HQ | pcr.F_PLAIN]
SHAPES = [None, {"ppt": 1, "wg": 64}, {"ppt": 8, "wg": 256}, {"ppt": 16, "wg": 64},
          {"ppt": 2, "wg": 1024}, {"ppt": 4, "wg": 128, "grid": 3}, {"ppt": 4, "run": 128},
          {"ppt": 2, "run": 6, "grid": 5}]


def dense_cloud(seed, n, W=48, H=32):
    """Many points per pixel, duplicated positions (equal keys) and a ragged
    tail relative to every tile size."""
    rng = np.random.default_rng(seed)
    m = synth.mvp((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, fovy=50.0)
    p = np.empty(n, synth.POINT_DTYPE)
    xyz = rng.uniform(-1.6, 1.6, (n, 3))
    xyz[n // 2:] = xyz[: n - n // 2]
    p["x"], p["y"], p["z"] = xyz.T
    p["rgba"] = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return p, m, W, H


@pytest.mark.parametrize("variant", BASIC_FORMS + HQ_FORMS)
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_dense_small(orc, variant, shape):
    pts, m, W, H = dense_cloud(1, 20_011)
    efb, eimg = oracle_frame(orc, pts, m, W, H, variant)
    fb, img = render_frame(upload(pts), m, W, H, variant, tune=SHAPES[shape])
    assert_same_fb(read_fb(fb, W, H, variant), efb, variant)
    assert np.array_equal(img, eimg)


@pytest.mark.parametrize("variant", [B, D, B | EZ | RD, HQ])
def test_sphere_1m_720p(orc, variant):
    """1M points on the unit sphere, random order, 1280x720."""
    pts = synth.sphere(1_000_000, seed=1)
    m = synth.sphere_view(1280, 720)
    efb, eimg = oracle_frame(orc, pts, m, 1280, 720, variant)
    fb, img = render_frame(upload(pts), m, 1280, 720, variant)
    assert_same_fb(read_fb(fb, 1280, 720, variant), efb, variant)
    assert np.array_equal(img, eimg)
    assert np.count_nonzero(img) > 100_000


@pytest.mark.parametrize("variant", [B, D, B | LDS | RD | EZ, HQ, HQ | LDS])
@pytest.mark.parametrize("order", ["scanline", "morton_shuffle"])
def test_terrain_2m_1080p(orc, variant, order):
    pts = synth.terrain(2_000_000, seed=2)
    if order == "morton_shuffle":
        pts = pts[orc.reorder(pts, 1, 128, 3)]
    m = synth.terrain_oblique(1920, 1080)
    efb, eimg = oracle_frame(orc, pts, m, 1920, 1080, variant)
    fb, img = render_frame(upload(pts), m, 1920, 1080, variant)
    assert_same_fb(read_fb(fb, 1920, 1080, variant), efb, variant)
    assert np.array_equal(img, eimg)


@pytest.mark.parametrize("variant", [D, HQ, B | LDS | RD, D | LDS | RD | EZ, HQ | LDS | RD | EZ])
@pytest.mark.parametrize("shape", [None, {"ppt": 16, "wg": 256}])
def test_ordered_and_scattered_tiles(orc, variant, shape):
    """One launch over ordered and scattered tiles: the first half of the
    cloud in scanline order (few pixels per tile, a full table) and the
    second half shuffled (a distinct pixel per point, table overflows), with
    and without the early depth test; the frame equals the oracle's."""
    pts = synth.terrain(2_000_000, seed=2)
    half = len(pts) // 2
    rng = np.random.default_rng(12)
    pts = np.concatenate([pts[:half], pts[half:][rng.permutation(len(pts) - half)]])
    m = synth.terrain_oblique(1280, 720)
    efb, eimg = oracle_frame(orc, pts, m, 1280, 720, variant)
    fb, img = render_frame(upload(pts), m, 1280, 720, variant, tune=shape)
    assert_same_fb(read_fb(fb, 1280, 720, variant), efb, variant)
    assert np.array_equal(img, eimg)


@pytest.mark.parametrize("variant", [B, D, B | RD, HQ, HQ | LDS])
def test_one_pixel_contention(orc, variant):
    """200k points on one view ray: maximal atomic contention on one pixel,
    a third of them at one shared depth (ties resolved by colour)."""
    n = 200_000
    rng = np.random.default_rng(3)
    p = np.empty(n, synth.POINT_DTYPE)
    z = rng.uniform(1.0, 3.0, n)
    z[::3] = 1.5
    p["x"], p["y"], p["z"] = 0.0, 0.0, z
    p["rgba"] = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    m = np.eye(4, dtype=np.float32).reshape(16).copy()
    m[14], m[15] = 1.0, 0.0
    W, H = 8, 8
    efb, eimg = oracle_frame(orc, p, m, W, H, variant)
    fb, img = render_frame(upload(p), m, W, H, variant)
    assert_same_fb(read_fb(fb, W, H, variant), efb, variant)
    assert np.array_equal(img, eimg)


@pytest.mark.parametrize("variant", [B, D, HQ])
def test_empty_and_single(orc, variant):
    pts, m, W, H = dense_cloud(5, 1)
    fb = pcr.alloc_fb(W, H, variant)
    _, img = render_frame(upload(pts), m, W, H, variant, fb=fb, n=0)
    assert not img.any()
    efb, eimg = oracle_frame(orc, pts, m, W, H, variant)
    fb, img = render_frame(upload(pts), m, W, H, variant)
    assert_same_fb(read_fb(fb, W, H, variant), efb, variant)
    assert np.array_equal(img, eimg)


@pytest.mark.parametrize("variant", [B, D, HQ])
def test_all_culled(orc, variant):
    pts = synth.terrain(300_000, seed=2)
    m = synth.terrain_away(320, 180)
    fb, img = render_frame(upload(pts), m, 320, 180, variant)
    assert not img.any()
    efb, _ = oracle_frame(orc, pts, m, 320, 180, variant)
    assert_same_fb(read_fb(fb, 320, 180, variant), efb, variant)


@pytest.mark.parametrize("variant", [B, D])
def test_accumulate(orc, variant):
    pts, m, W, H = dense_cloud(6, 30_000)
    d = upload(pts)
    fb = pcr.alloc_fb(W, H, variant)
    pcr.fb_clear(fb, W, H, variant)
    pcr.render(d[:12_345], m, W, H, variant, fb)
    pcr.render(d[12_345:], m, W, H, variant, fb)
    efb, _ = oracle_frame(orc, pts, m, W, H, variant)
    import torch
    torch.cuda.synchronize()
    assert_same_fb(read_fb(fb, W, H, variant), efb, variant)


def test_hq_split_passes(orc):
    """Depth pass over two buffers, then colour pass over both = HQ of the union."""
    pts, m, W, H = dense_cloud(7, 40_000)
    d = upload(pts)
    fb = pcr.alloc_fb(W, H, HQ)
    pcr.fb_clear(fb, W, H, HQ)
    for part in (d[:17_000], d[17_000:]):
        pcr.render(part, m, W, H, HQ | pcr.F_HQ_DEPTH, fb)
    for part in (d[:17_000], d[17_000:]):
        pcr.render(part, m, W, H, HQ | pcr.F_HQ_COLOR | pcr.F_LDS, fb)
    img = pcr.resolve(fb, W, H, HQ).cpu().numpy().view(np.uint32)
    efb, eimg = oracle_frame(orc, pts, m, W, H, HQ)
    assert_same_fb(read_fb(fb, W, H, HQ), efb, HQ)
    assert np.array_equal(img, eimg)


def test_odd_sizes(orc):
    """1x1, a single row and a single column; pixel counts that are odd."""
    pts, _, _, _ = dense_cloud(8, 5000)
    for W, H in [(1, 1), (333, 1), (1, 257), (17, 13)]:
        m = synth.mvp((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, fovy=50.0)
        for variant in (B, D, HQ):
            efb, eimg = oracle_frame(orc, pts, m, W, H, variant)
            fb, img = render_frame(upload(pts), m, W, H, variant)
            assert_same_fb(read_fb(fb, W, H, variant), efb, variant)
            assert np.array_equal(img, eimg)


def test_oversized_lds_tile_is_rejected():
    pts, m, W, H = dense_cloud(9, 100)
    fb = pcr.alloc_fb(W, H, HQ)
    with pytest.raises(pcr.PcrError) as e:
        pcr.render(upload(pts), m, W, H, HQ | LDS, fb, tune={"ppt": 16, "wg": 1024})
    assert e.value.code == pcr.EINVAL


@pytest.mark.parametrize("shape", [None, {"run": 4}, {"run": 32}, {"run": 128}, {"ppt": 8, "wg": 256},
                                   {"ppt": 16, "wg": 128}, {"ppt": 1, "run": 0}])
def test_basic_lane_mappings(orc, shape):
    """The basic kernel's lane mappings (adaptive default, fixed runs) on a
    cloud whose first part repeats each position over runs of consecutive
    points (consecutive points share pixels: the adaptive mapping switches to
    runs) and whose second part is in random order (it stays interleaved);
    51,203 points, so tiles and sub-tiles end ragged."""
    rng = np.random.default_rng(7)
    W, H = 96, 64
    m = synth.mvp((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, fovy=50.0)
    n1, n2 = 40_000, 11_203
    p = np.empty(n1 + n2, synth.POINT_DTYPE)
    base = rng.uniform(-1.6, 1.6, (n1 // 8, 3))
    xyz = np.repeat(base, 8, axis=0)
    xyz += rng.normal(0.0, 1e-4, xyz.shape)
    p["x"][:n1], p["y"][:n1], p["z"][:n1] = xyz.T
    p["x"][n1:], p["y"][n1:], p["z"][n1:] = rng.uniform(-1.6, 1.6, (n2, 3)).T
    p["rgba"] = rng.integers(0, 2**32, len(p), dtype=np.uint64).astype(np.uint32)
    efb, eimg = oracle_frame(orc, p, m, W, H, B)
    fb, img = render_frame(upload(p), m, W, H, B, tune=shape)
    assert_same_fb(read_fb(fb, W, H, B), efb, B)
    assert np.array_equal(img, eimg)
