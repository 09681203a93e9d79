"""GPU parity on hostile float inputs: NaN, infinities, signed zeros,
subnormal coordinates, clip w in the reciprocal's slow ranges (below 2^-125,
above 2^126, and overflowing to infinity), w exactly zero, and
dyadic points that land exactly on pixel and viewport edges.  Every variant,
the chunked path and both batch modes must give the oracle's framebuffer and
image bit for bit (the viewport test, the culling of NaN and the early
wavefront cull all decide in float32 on both sides)."""
import numpy as np
import pytest

from gpu_util import assert_same_fb, hq_depth_bytes, oracle_frame, read_fb, render_frame, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu

B, D, HQ = pcr.BASIC, pcr.DEDUP, pcr.HQ
EZ, RD, LDS = pcr.F_EARLYZ, pcr.F_REDUCE, pcr.F_LDS
VARIANTS = [B, D, B | EZ | RD, B | LDS | EZ, D | pcr.F_PLAIN, HQ, HQ | LDS | RD | EZ, HQ | pcr.F_PLAIN]

SPECIAL = np.array([0.0, -0.0, 1.0, -1.0, 0.5, np.nan, -np.nan, np.inf, -np.inf, 1e-45, -1e-45, 1e-40,
                    2.0 ** -126, 3.4e38, -3.4e38, 1e38, 65504.0, 2.0 ** -20], np.float32)


def _m(rows):
    return np.asarray(rows, np.float64).astype(np.float32).reshape(16)


def matrices(W, H):
    s_lo, s_hi = 2.0 ** -126, 2.0 ** 126
    return {
        # a camera at distance 3 looking at the origin
        "perspective": synth.mvp((0.0, 0.0, 3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H),
        # clip (x, y, z): with z = 1 the dyadic points fall exactly on pixel edges
        "dyadic": _m([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 0], [0, 0, 1, 0]]),
        # clip coordinates subnormal for |x| < 1; w around 2^-125, the reciprocal's low slow range
        "tiny_w": _m([[s_lo, 0, 0, 0], [0, s_lo, 0, 0], [0, 0, 0, 0], [0, 0, s_lo, 0]]),
        # w above 2^126 for z > 1 (the high slow range); infinite for the large special values
        "huge_w": _m([[s_hi, 0, 0, 0], [0, s_hi, 0, 0], [0, 0, 0, 0], [0, 0, s_hi, 0]]),
        # w = z - 1: exactly +0 at z = 1, negative below
        "w_through_zero": _m([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 0], [0, 0, 1, -1]]),
    }


def special_cloud(seed, n):
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-1.2, 1.2, (n, 3)).astype(np.float32)
    xyz[:, 2] = rng.uniform(0.25, 2.5, n).astype(np.float32)
    k = n // 4                                   # dyadic points on pixel edges, z = 1
    xyz[:k, 0] = rng.integers(-40, 41, k) / np.float32(32.0)
    xyz[:k, 1] = rng.integers(-40, 41, k) / np.float32(32.0)
    xyz[:k, 2] = 1.0
    hit = rng.random((n, 3)) < 0.08               # special values anywhere
    xyz[hit] = rng.choice(SPECIAL, int(hit.sum()))
    p = np.empty(n, synth.POINT_DTYPE)
    p["x"], p["y"], p["z"] = xyz.T
    p["rgba"] = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return p


@pytest.fixture(scope="module")
def cloud():
    pts = special_cloud(17, 40_009)
    return pts, upload(pts)


@pytest.mark.parametrize("size", [(64, 48), (37, 5)])
@pytest.mark.parametrize("name", ["perspective", "dyadic", "tiny_w", "huge_w", "w_through_zero"])
def test_hostile_floats_every_variant(orc, cloud, name, size):
    pts, d = cloud
    W, H = size
    m = matrices(W, H)[name]
    drawn = 0
    for variant in VARIANTS:
        efb, eimg = oracle_frame(orc, pts, m, W, H, variant)
        fb, img = render_frame(d, m, W, H, variant)
        assert_same_fb(read_fb(fb, W, H, variant), efb, variant)
        assert np.array_equal(img, eimg), variant
        drawn = max(drawn, int(np.count_nonzero(eimg)))
    assert drawn > 0, "no point of the cloud lands in this view"


@pytest.mark.parametrize("name", ["dyadic", "tiny_w", "huge_w", "w_through_zero"])
def test_hostile_floats_packed_hq(orc, cloud, name):
    import torch
    pts, d = cloud
    W, H = 64, 48
    m = matrices(W, H)[name]
    v = HQ | pcr.F_HQ_PACKED
    eD, eP = orc.render_hq_packed(pts, m, W, H)
    fb = pcr.alloc_fb(W, H, v)
    pcr.fb_clear(fb, W, H, v)
    pcr.render(d, m, W, H, v, fb)
    img = pcr.resolve(fb, W, H, v)
    torch.cuda.synchronize()
    raw = fb.cpu().numpy().view(np.uint8)
    assert np.array_equal(raw[: 4 * W * H].view(np.uint32), eD)
    off = hq_depth_bytes(W, H)
    assert np.array_equal(raw[off: off + 8 * W * H].view(np.uint64), eP)
    assert np.array_equal(img.cpu().numpy().view(np.uint32), orc.resolve_hq_packed(eP, W, H))


@pytest.mark.parametrize("variant", [D, HQ])
def test_hostile_floats_chunked(orc, cloud, variant):
    import torch
    pts, d = cloud
    W, H = 64, 48
    rng = np.random.default_rng(5)
    for name, m in matrices(W, H).items():
        efb, eimg = oracle_frame(orc, pts, m, W, H, variant)
        cuts = np.sort(rng.choice(np.arange(1, len(pts)), 60, replace=False))
        offs = np.concatenate([[0], cuts, [len(pts)]])
        table = [(d.data_ptr() + 16 * int(a), int(b - a)) for a, b in zip(offs[:-1], offs[1:])]
        rng.shuffle(table)
        fb = pcr.alloc_fb(W, H, variant)
        pcr.fb_clear(fb, W, H, variant)
        pcr.render_chunks(pcr.chunk_table(table), len(table), m, W, H, variant, fb)
        img = pcr.resolve(fb, W, H, variant)
        torch.cuda.synchronize()
        assert_same_fb(read_fb(fb, W, H, variant), efb, variant)
        assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg), name


@pytest.mark.parametrize("tune", [{"group": 1}, {"ppt": 8, "group": 4}])
def test_hostile_floats_batched(orc, cloud, tune):
    import torch
    pts, d = cloud
    views = []
    for W, H in ((64, 48), (37, 5)):
        for name, m in matrices(W, H).items():
            for variant in (B, HQ):
                views.append((name, m, W, H, variant))
    plan = pcr.BatchPlan(d, capacity=len(views), tune=tune)
    bufs, pv = [], []
    for _, m, W, H, variant in views:
        fb = pcr.alloc_fb(W, H, variant)
        img = torch.zeros(W * H, dtype=torch.int32, device="cuda")
        bufs.append((fb, img))
        pv.append(pcr.make_view(m, W, H, variant, fb, img))
    plan.launch(pv)
    torch.cuda.synchronize()
    for (name, m, W, H, variant), (fb, img) in zip(views, bufs):
        efb, eimg = oracle_frame(orc, pts, m, W, H, variant)
        assert_same_fb(read_fb(fb, W, H, variant), efb, variant)
        assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg), (name, W, H, variant)
    plan.close()


@pytest.mark.parametrize("order", [pcr.ORDER_MORTON, pcr.ORDER_MORTON_SHUFFLE, pcr.ORDER_SHUFFLE])
def test_reorder_of_non_finite_coordinates_is_a_permutation(orc, cloud, order):
    """Coordinates outside the reorder's domain (NaN, infinities) leave the
    Morton order unspecified, but the output is still a permutation of the
    input with out = in[perm]; the shuffled order, which ignores positions,
    still equals the oracle's."""
    import torch
    from gpu_util import download_points
    pts, d = cloud
    out, perm = pcr.reorder(d, order, 128, 9)
    torch.cuda.synchronize()
    p = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(p), np.arange(len(pts)))
    assert np.array_equal(download_points(out).view(np.uint32).reshape(-1, 4),
                          pts[p].view(np.uint32).reshape(-1, 4))
    if order == pcr.ORDER_SHUFFLE:
        assert np.array_equal(p, orc.reorder(pts, order, 128, 9))
