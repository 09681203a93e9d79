"""GPU parity of the single-atomic HQ form (PCR_F_HQ_PACKED: one 18-18-18-10
word per pixel) against the CPU oracle, bit for bit: depth buffer, packed
words and images, on every update path and launch shape, in the exact range
(at most 1023 points per pixel) and past it, where the fields wrap and carry
exactly as the oracle's modular sums do."""
import numpy as np
import pytest

from gpu_util import hq_depth_bytes, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu

PK = pcr.HQ | pcr.F_HQ_PACKED
PATHS = [PK, PK | pcr.F_LDS, PK | pcr.F_LDS | pcr.F_REDUCE, PK | pcr.F_LDS | pcr.F_EARLYZ, PK | pcr.F_PLAIN]
SHAPES = [None, {"ppt": 1, "wg": 64}, {"ppt": 16, "wg": 256}, {"ppt": 4, "wg": 1024}, {"ppt": 8, "grid": 5}]


def read_packed(fb, W, H):
    raw = fb.cpu().numpy().view(np.uint8)
    D = raw[: 4 * W * H].view(np.uint32).copy()
    off = hq_depth_bytes(W, H)
    P = raw[off: off + 8 * W * H].view(np.uint64).copy()
    return D, P


def gpu_packed(pts_dev, m, W, H, variant, tune=None):
    import torch
    fb = pcr.alloc_fb(W, H, variant)
    pcr.fb_clear(fb, W, H, variant)
    pcr.render(pts_dev, m, W, H, variant, fb, tune=tune)
    img = pcr.resolve(fb, W, H, variant)
    torch.cuda.synchronize()
    return fb, img.cpu().numpy().view(np.uint32)


def check(orc, pts, m, W, H, variant, tune=None, dev=None):
    eD, eP = orc.render_hq_packed(pts, m, W, H)
    eimg = orc.resolve_hq_packed(eP, W, H)
    fb, img = gpu_packed(upload(pts) if dev is None else dev, m, W, H, variant, tune)
    D, P = read_packed(fb, W, H)
    assert np.array_equal(D, eD)
    bad = np.nonzero(P != eP)[0]
    assert len(bad) == 0, (len(bad), bad[:4], P[bad[:4]], eP[bad[:4]])
    assert np.array_equal(img, eimg)
    return eP, img


def dense_cloud(seed, n, W=48, H=32):
    rng = np.random.default_rng(seed)
    m = synth.mvp((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, fovy=50.0)
    p = np.empty(n, synth.POINT_DTYPE)
    xyz = rng.uniform(-1.6, 1.6, (n, 3))
    xyz[n // 2:] = xyz[: n - n // 2]
    p["x"], p["y"], p["z"] = xyz.T
    p["rgba"] = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return p, m, W, H


@pytest.mark.parametrize("variant", PATHS)
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_dense_small(orc, variant, shape):
    pts, m, W, H = dense_cloud(1, 20_011)
    check(orc, pts, m, W, H, variant, SHAPES[shape])


def test_equals_two_word_hq_within_the_bound(orc):
    """1M sphere points at 1280x720: no pixel takes 1024 points, so the packed
    image equals the two-word HQ image."""
    pts = synth.sphere(1_000_000, seed=1)
    m = synth.sphere_view(1280, 720)
    _, RG, BA = orc.render_hq(pts, m, 1280, 720)
    assert int((BA & np.uint64(0xFFFFFFFF)).max()) <= 1023
    _, img = check(orc, pts, m, 1280, 720, PK)
    assert np.array_equal(img, orc.resolve_hq(RG, BA, 1280, 720))


@pytest.mark.parametrize("variant", [PK, PK | pcr.F_PLAIN, PK | pcr.F_LDS])
@pytest.mark.parametrize("count", [1023, 1024, 1025, 200_000])
def test_past_the_bound(orc, variant, count):
    """Many points at one pixel and one depth: the packed word wraps and
    carries like the oracle's sum modulo 2^64 (1024 points resolve empty)."""
    rng = np.random.default_rng(count)
    p = np.empty(count, synth.POINT_DTYPE)
    p["x"], p["y"], p["z"] = 0.0, 0.0, 1.5
    p["rgba"] = rng.integers(0, 2**32, count, dtype=np.uint64).astype(np.uint32)
    m = np.eye(4, dtype=np.float32).reshape(16).copy()
    m[14], m[15] = 1.0, 0.0
    W, H = 8, 8
    eP, img = check(orc, p, m, W, H, variant)
    if count == 1024:
        assert not img.any()
    if count == 1023:
        assert img[4 * W + 4] != 0


@pytest.mark.parametrize("order", ["scanline", "morton_shuffle"])
def test_terrain_2m_1080p(orc, order):
    pts = synth.terrain(2_000_000, seed=2)
    if order == "morton_shuffle":
        pts = pts[orc.reorder(pts, 1, 128, 3)]
    check(orc, pts, synth.terrain_oblique(1920, 1080), 1920, 1080, PK)


def test_split_passes_chunks_and_depth_resolve(orc):
    """Depth pass and colour pass as two calls, the same frame from a chunk
    table, and the colour of the depth resolve equal the oracle's."""
    import torch
    pts = synth.terrain(600_000, seed=9)
    W, H = 640, 360
    m = synth.terrain_oblique(W, H)
    eD, eP = orc.render_hq_packed(pts, m, W, H)
    eimg = orc.resolve_hq_packed(eP, W, H)
    dev = upload(pts)
    fb = pcr.alloc_fb(W, H, PK)
    pcr.fb_clear(fb, W, H, PK)
    pcr.render(dev, m, W, H, PK | pcr.F_HQ_DEPTH, fb)
    pcr.render(dev, m, W, H, PK | pcr.F_HQ_COLOR, fb)
    torch.cuda.synchronize()
    D, P = read_packed(fb, W, H)
    assert np.array_equal(D, eD) and np.array_equal(P, eP)
    sizes = np.random.default_rng(4).integers(1, 5000, 400)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    offs = offs[offs <= len(pts)]
    table = [(dev.data_ptr() + 16 * int(a), int(b - a)) for a, b in zip(offs[:-1], offs[1:])]
    table.append((dev.data_ptr() + 16 * int(offs[-1]), len(pts) - int(offs[-1])))
    fb2 = pcr.alloc_fb(W, H, PK)
    pcr.fb_clear(fb2, W, H, PK)
    pcr.render_chunks(pcr.chunk_table(table), len(table), m, W, H, PK, fb2)
    rgba = torch.empty(W * H, dtype=torch.int32, device="cuda")
    depth, _ = pcr.resolve_depth(fb2, W, H, PK, pcr.DEPTH_LINEAR, rgba=rgba)
    torch.cuda.synchronize()
    D2, P2 = read_packed(fb2, W, H)
    assert np.array_equal(D2, eD) and np.array_equal(P2, eP)
    assert np.array_equal(rgba.cpu().numpy().view(np.uint32), eimg)
    want = orc.resolve_depth_hq(eD, W, H)
    assert np.array_equal(depth.cpu().numpy().view(np.uint32), want.view(np.uint32))


def test_rejected_in_batch_views():
    pts = upload(synth.sphere(10_000, seed=1))
    W, H = 64, 64
    fb = pcr.alloc_fb(W, H, pcr.HQ)
    import torch
    img = torch.empty(W * H, dtype=torch.int32, device="cuda")
    plan = pcr.BatchPlan(pts, 2)
    try:
        with pytest.raises(pcr.PcrError) as e:
            plan.launch([pcr.make_view(synth.sphere_view(W, H), W, H, PK, fb, img)])
        assert e.value.code == pcr.EUNSUPPORTED
    finally:
        plan.close()
