"""Helpers for the GPU tests: upload inputs, run the library, read results back."""
from __future__ import annotations

import numpy as np

from paper_2104_07526_amd import pcr, synth


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a GPU (run them with -m gpu on an MI355X)")
    return torch.device("cuda", 0)


def upload(points):
    import torch
    a = np.ascontiguousarray(points)
    assert a.dtype == synth.POINT_DTYPE
    t = torch.from_numpy(a.view(np.int32).reshape(-1, 4))
    return t.to(device())


def download_points(t):
    return t.cpu().numpy().reshape(-1).view(synth.POINT_DTYPE)


def hq_depth_bytes(W, H):
    return (4 * W * H + 255) // 256 * 256


def read_fb(fb, W, H, variant):
    """Basic: u64[W*H]; HQ: (D u32[W*H], RG u64[W*H], BA u64[W*H])."""
    raw = fb.cpu().numpy().view(np.uint8)
    if (variant & 0xFF) != pcr.HQ:
        return raw[: 8 * W * H].view(np.uint64).copy()
    D = raw[: 4 * W * H].view(np.uint32).copy()
    off = hq_depth_bytes(W, H)
    S = raw[off: off + 16 * W * H].view(np.uint64)
    return D, S[0::2].copy(), S[1::2].copy()


def render_frame(pts_dev, m, W, H, variant, tune=None, clear=True, fb=None, n=None):
    """clear + render + resolve on the current stream; returns (fb, image)."""
    import torch
    if fb is None:
        fb = pcr.alloc_fb(W, H, variant)
    if clear:
        pcr.fb_clear(fb, W, H, variant)
    pcr.render(pts_dev, m, W, H, variant, fb, tune=tune, n=n)
    img = pcr.resolve(fb, W, H, variant)
    torch.cuda.synchronize()
    return fb, img.cpu().numpy().view(np.uint32)


def oracle_frame(orc, pts, m, W, H, variant):
    """The oracle's framebuffer (as read_fb returns it) and image."""
    if (variant & 0xFF) == pcr.HQ:
        D, RG, BA = orc.render_hq(pts, m, W, H)
        return (D, RG, BA), orc.resolve_hq(RG, BA, W, H)
    fb = orc.render_basic(pts, m, W, H)
    return fb, orc.resolve_basic(fb, W, H)


def assert_same_fb(got, exp, variant):
    if (variant & 0xFF) == pcr.HQ:
        for name, g, e in zip(("depth", "RG", "BA"), got, exp):
            bad = np.nonzero(g != e)[0]
            assert len(bad) == 0, f"{name}: {len(bad)} pixels differ, first {bad[:5]}: {g[bad[:5]]} vs {e[bad[:5]]}"
    else:
        bad = np.nonzero(got != exp)[0]
        assert len(bad) == 0, f"{len(bad)} pixels differ, first {bad[:5]}: {got[bad[:5]]} vs {exp[bad[:5]]}"
