"""GPU vertex orders (Morton, shuffled Morton, shuffled) against the oracle:
bit-exact permutations and reordered buffers; images independent of order."""
import numpy as np
import pytest

from gpu_util import download_points, oracle_frame, render_frame, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu

ORDERS = [pcr.ORDER_MORTON, pcr.ORDER_MORTON_SHUFFLE, pcr.ORDER_SHUFFLE]


def cloud(n, seed=0, dup=True):
    rng = np.random.default_rng(seed)
    p = np.empty(n, synth.POINT_DTYPE)
    xyz = rng.uniform(-3.0, 7.0, (n, 3)) * np.array([1.0, 0.5, 0.25])
    if dup and n > 4:
        xyz[n - n // 4:] = xyz[: n // 4]          # equal codes: stability matters
    p["x"], p["y"], p["z"] = xyz.T
    p["rgba"] = np.arange(n, dtype=np.uint32)
    return p


def gpu_reorder(pts, order, batch=128, seed=0):
    import torch
    d = upload(pts)
    out, perm = pcr.reorder(d, order, batch=batch, seed=seed)
    torch.cuda.synchronize()
    return download_points(out), perm.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("n", [1, 2, 127, 128, 129, 4095, 4096, 4097, 8191, 8192, 8193, 16_385, 65_537, 300_001])
def test_perm_matches_oracle(orc, order, n):
    pts = cloud(n, seed=n)
    exp = orc.reorder(pts, order, 128, 77)
    out, perm = gpu_reorder(pts, order, 128, 77)
    assert np.array_equal(perm, exp)
    assert np.array_equal(out.view(np.uint32), pts[exp].view(np.uint32))


@pytest.mark.parametrize("batch", [1, 3, 128, 1000, 5000])
def test_batch_sizes(orc, batch):
    pts = cloud(4321, seed=5)
    exp = orc.reorder(pts, pcr.ORDER_MORTON_SHUFFLE, batch, 9)
    _, perm = gpu_reorder(pts, pcr.ORDER_MORTON_SHUFFLE, batch, 9)
    assert np.array_equal(perm, exp)


def test_terrain_2m(orc):
    pts = synth.terrain(2_000_000, seed=2)
    for order in ORDERS:
        exp = orc.reorder(pts, order, 128, 3)
        _, perm = gpu_reorder(pts, order, 128, 3)
        assert np.array_equal(perm, exp), order


def test_degenerate_boxes(orc):
    """All points equal (zero-size box), a flat cloud, negative zeros."""
    n = 5000
    p = cloud(n, seed=1, dup=False)
    flat = p.copy()
    flat["z"] = 0.0
    flat["z"][::2] = -0.0
    same = p.copy()
    same["x"], same["y"], same["z"] = 1.5, -2.0, 0.0
    for q in (flat, same):
        for order in ORDERS:
            exp = orc.reorder(q, order, 128, 4)
            _, perm = gpu_reorder(q, order, 128, 4)
            assert np.array_equal(perm, exp)


def test_empty_and_scratch_errors():
    import torch
    d = upload(cloud(1000))
    need = pcr.reorder_scratch_bytes(1000, pcr.ORDER_MORTON_SHUFFLE, 128)
    small = torch.empty(need - 256, dtype=torch.uint8, device=d.device)
    with pytest.raises(pcr.PcrError) as e:
        pcr.reorder(d, pcr.ORDER_MORTON_SHUFFLE, scratch=small)
    assert e.value.code == pcr.ENOMEM
    out, perm = pcr.reorder(d[:0], pcr.ORDER_MORTON)
    assert out.numel() == 0


@pytest.mark.parametrize("variant", [pcr.BASIC, pcr.DEDUP, pcr.HQ])
def test_image_independent_of_order(orc, variant):
    pts = synth.terrain(1_000_000, seed=2)
    m = synth.terrain_oblique(640, 360)
    _, ref = oracle_frame(orc, pts, m, 640, 360, variant)
    d = upload(pts)
    for order in ORDERS:
        out, _ = pcr.reorder(d, order, seed=8)
        _, img = render_frame(out, m, 640, 360, variant)
        assert np.array_equal(img, ref), order
