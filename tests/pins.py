"""Pins of the CPU oracle against facts that do not come from the oracle.

Each ``check_*`` takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with a closed form, a hand-derived value, an error bound of
exact arithmetic, a brute-force gather, a published test vector or an invariant
of the method.  The same checks run against deliberately broken builds of the
oracle (tests/test_oracle_mutants.py) to show that each plausible mistake is
caught by at least one of them.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from paper_2104_07526_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FULL = 0xFFFFFFFFFFFFFFFF


def f32bits(v: float) -> int:
    return int(np.float32(v).view(np.uint32))


def bits2f(u: int) -> float:
    return float(np.uint32(u).view(np.float32))


def make_points(xyz, rgba):
    p = np.empty(len(xyz), synth.POINT_DTYPE)
    xyz = np.asarray(xyz, np.float64).reshape(-1, 3)
    p["x"], p["y"], p["z"] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    p["rgba"] = np.asarray(rgba, np.uint32)
    return p


def identity(**kw):
    m = np.eye(4, dtype=np.float32).reshape(16)
    for k, v in kw.items():
        m[int(k[1:])] = v
    return m


# ---------------------------------------------------------------------------
# Projection (Sec. 3.1; the pixel convention is this project's reading)
# ---------------------------------------------------------------------------

def check_hand_cases(orc):
    """Single points whose pixel and depth follow by hand (tests/golden)."""
    with open(os.path.join(GOLDEN, "hand_projection.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        m = np.zeros(16, np.float32)
        m[:] = c["mvp"]
        got = orc.project(m, c["W"], c["H"], *c["xyz"])
        if c["expect"] is None:
            assert got is None, (c["name"], got)
        else:
            assert got is not None, c["name"]
            assert got[0] == c["expect"]["pid"], (c["name"], got)
            assert got[1] == int(c["expect"]["depth_bits"], 16), (c["name"], hex(got[1]))


def _camera_cloud(seed, n=4000):
    rng = np.random.default_rng(seed)
    W, H = 160, 90
    m = synth.mvp(rng.uniform(-4, 4, 3) + np.array([0, 0, 6.0]), rng.uniform(-0.5, 0.5, 3),
                  (0.0, 1.0, 0.0), W, H, fovy=float(rng.uniform(30, 90)))
    pts = make_points(rng.uniform(-2.0, 2.0, (n, 3)), rng.integers(0, 2**32, n, dtype=np.uint64))
    return pts, m, W, H


def check_projection_fp64(orc):
    """Against exact arithmetic: the float32 pipeline may only differ from the
    real-number result by a few units in the last place, so away from pixel
    edges the pixel must equal floor() of the float64 result, and the depth
    must lie within the summation error bound of the float64 depth."""
    for seed in range(4):
        pts, m, W, H = _camera_cloud(seed)
        pid, d = orc.project_all(pts, m, W, H)
        M = m.astype(np.float64).reshape(4, 4)
        P = np.stack([pts["x"], pts["y"], pts["z"], np.ones(len(pts), np.float32)], 1).astype(np.float64)
        clip = P @ M.T
        w = clip[:, 3]
        mag = np.abs(P * M[3][None, :]).sum(1)
        eps = 2.0 ** -24
        front = w > 8 * eps * mag
        fx = (clip[:, 0] / np.where(front, w, 1.0) + 1.0) * (W / 2)
        fy = (clip[:, 1] / np.where(front, w, 1.0) + 1.0) * (H / 2)
        tol = 1e-3
        safe = front & (np.abs(fx - np.round(fx)) > tol) & (np.abs(fy - np.round(fy)) > tol)
        inside = safe & (fx > 0) & (fx < W) & (fy > 0) & (fy < H)
        outside = safe & ~((fx > -tol) & (fx < W + tol) & (fy > -tol) & (fy < H + tol))
        assert inside.sum() > 500, "too few visible points for the check"
        exp = (np.floor(fy[inside]).astype(np.int64) * W + np.floor(fx[inside]).astype(np.int64))
        assert np.array_equal(pid[inside].astype(np.int64), exp)
        assert np.all(pid[outside] == 0xFFFFFFFF)
        assert np.all(pid[~front & (w < 0)] == 0xFFFFFFFF)
        dep = d[inside].view(np.float32).astype(np.float64)
        assert np.all(np.abs(dep - w[inside]) <= 4 * eps * mag[inside] + 1e-30)


def check_projection_dyadic(orc):
    """With small dyadic inputs every float32 product and sum is exact, so the
    depth equals the exact row-3 dot product and the pixel follows from one
    correctly rounded reciprocal (exact for power-of-two depths)."""
    rng = np.random.default_rng(11)
    W, H = 64, 32
    for _ in range(200):
        m = (rng.integers(-8, 9, 16) / 4.0).astype(np.float32)
        m[15] = 8.0
        xyz = rng.integers(-8, 9, 3) / 8.0
        w = float(m[12:15].astype(np.float64) @ xyz + m[15])
        if w <= 0:
            assert orc.project(m, W, H, *xyz) is None
            continue
        got = orc.project(m, W, H, *xyz)
        if got is None:
            # Culled only if the exact position is outside (or on the open edge).
            cx = float(m[0:3].astype(np.float64) @ xyz + m[3])
            cy = float(m[4:7].astype(np.float64) @ xyz + m[7])
            fx = (cx / w + 1) * W / 2
            fy = (cy / w + 1) * H / 2
            assert not (0.01 < fx < W - 0.01 and 0.01 < fy < H - 0.01), (m, xyz)
            continue
        assert got[1] == f32bits(w)
        if w in (1.0, 2.0, 4.0, 8.0, 16.0):
            cx = float(m[0:3].astype(np.float64) @ xyz + m[3])
            cy = float(m[4:7].astype(np.float64) @ xyz + m[7])
            fx = (cx / w + 1) * W / 2
            fy = (cy / w + 1) * H / 2
            assert got[0] == int(math.floor(fy)) * W + int(math.floor(fx))


def check_projection_rounding(orc):
    """Each step is one binary32 operation with round-to-nearest and no fused
    multiply-add: numpy's float32 ufuncs, one array operation per step, give
    the same bits (this pins the rounding, the formula is pinned above)."""
    for seed in range(3):
        pts, m, W, H = _camera_cloud(100 + seed, n=20000)
        pid, d = orc.project_all(pts, m, W, H)
        f = np.float32
        x, y, z = pts["x"], pts["y"], pts["z"]
        row = lambda r: ((m[4 * r] * x + m[4 * r + 1] * y) + m[4 * r + 2] * z) + m[4 * r + 3]  # noqa: E731
        cx, cy, cw = row(0), row(1), row(3)
        ok = cw > f(0)
        rw = f(1) / np.where(ok, cw, f(1))
        fx = (cx * rw + f(1)) * (f(0.5) * f(W))
        fy = (cy * rw + f(1)) * (f(0.5) * f(H))
        ok &= (fx >= 0) & (fx < f(W)) & (fy >= 0) & (fy < f(H))
        assert np.array_equal(pid != 0xFFFFFFFF, ok)
        exp = fy[ok].astype(np.uint32) * np.uint32(W) + fx[ok].astype(np.uint32)
        assert np.array_equal(pid[ok], exp)
        assert np.array_equal(d[ok], cw[ok].view(np.uint32))


# ---------------------------------------------------------------------------
# Basic render + resolve (Sec. 3.1)
# ---------------------------------------------------------------------------

def brute_force_basic(pid, dbits, rgba, W, H):
    """Per-pixel gather: for every pixel scan all points and keep the smallest
    (depth, colour) pair -- the opposite loop nest to the oracle's scatter."""
    fb = np.full(W * H, FULL, dtype=np.uint64)
    for p in range(W * H):
        hit = np.nonzero(pid == p)[0]
        best = None
        for i in hit:
            k = (int(dbits[i]) << 32) | int(rgba[i])
            if best is None or k < best:
                best = k
        if best is not None:
            fb[p] = best
    return fb


def _dense_tiny_cloud(seed, n=1500):
    """A tiny cloud in front of a 24x16 view, with many points per pixel and
    deliberate depth ties."""
    rng = np.random.default_rng(seed)
    W, H = 24, 16
    m = synth.mvp((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, fovy=50.0)
    xyz = rng.uniform(-1.5, 1.5, (n, 3))
    xyz[n // 2:, :] = xyz[: n - n // 2, :]        # exact duplicates: same pixel, same depth
    rgba = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    return make_points(xyz, rgba), m, W, H


def check_basic_brute_force(orc):
    for seed in range(3):
        pts, m, W, H = _dense_tiny_cloud(seed)
        pid, d = orc.project_all(pts, m, W, H)
        fb = orc.render_basic(pts, m, W, H)
        bf = brute_force_basic(pid, d, pts["rgba"], W, H)
        assert np.array_equal(fb, bf)
        assert (fb != FULL).sum() > W * H // 3


def check_basic_permutation(orc):
    pts, m, W, H = _dense_tiny_cloud(7)
    ref = orc.render_basic(pts, m, W, H)
    rng = np.random.default_rng(3)
    for _ in range(3):
        assert np.array_equal(orc.render_basic(pts[rng.permutation(len(pts))], m, W, H), ref)


def check_basic_accumulate(orc):
    """Rendering two halves into one cleared framebuffer equals rendering all."""
    pts, m, W, H = _dense_tiny_cloud(8)
    fb = orc.render_basic(pts[:700], m, W, H)
    fb = orc.render_basic(pts[700:], m, W, H, fb=fb)
    assert np.array_equal(fb, orc.render_basic(pts, m, W, H))


def check_basic_closest_wins(orc):
    """Points on one view ray: the nearest one's colour is shown, whatever
    the colours (a larger colour word at smaller depth must still win)."""
    W, H = 8, 8
    m = identity(m14=1.0, m15=0.0)   # clip w = z
    zs = [3.0, 0.5, 2.0, 0.75]
    cols = [0x00000001, 0xFFFFFFFF, 0x00000002, 0x00000003]
    pts = make_points([(0.0, 0.0, z) for z in zs], cols)
    fb = orc.render_basic(pts, m, W, H)
    out = orc.resolve_basic(fb, W, H)
    p = 4 * W + 4
    assert fb[p] == (f32bits(0.5) << 32) | 0xFFFFFFFF
    assert out[p] == 0xFFFFFFFF
    assert np.count_nonzero(out) == 1
    # Equal depth: the smaller colour word wins (the low half of the key).
    pts = make_points([(0.0, 0.0, 1.0), (0.0, 0.0, 1.0)], [0x0A0B0C0D, 0x0A0B0C0C])
    out = orc.resolve_basic(orc.render_basic(pts, m, W, H), W, H)
    assert out[p] == 0x0A0B0C0C


def check_resolve_basic(orc):
    fb = np.array([FULL, 0x3F800000_12345678, 0x0000000F_00000000, 0xFFFFFFFF_00000001], np.uint64)
    assert orc.resolve_basic(fb, 2, 2).tolist() == [0, 0x12345678, 0, 1]


# ---------------------------------------------------------------------------
# High-quality blend (Sec. 3.5)
# ---------------------------------------------------------------------------

def _hq_image(orc, pts, m, W, H):
    D, RG, BA = orc.render_hq(pts, m, W, H)
    return orc.resolve_hq(RG, BA, W, H), D, RG, BA


def check_hq_special_cases(orc):
    W, H = 8, 8
    m = identity(m14=1.0, m15=0.0)   # clip w = z, pixel (4,4) for x = y = 0
    p = 4 * W + 4
    rgb = lambda r, g, b: int(synth.pack_rgba(r, g, b))  # noqa: E731
    # One point per pixel: HQ shows the point's RGB with alpha 255.
    out, D, RG, BA = _hq_image(orc, make_points([(0, 0, 2.0)], [rgb(10, 20, 30) & 0x00FFFFFF]), m, W, H)
    assert out[p] == rgb(10, 20, 30)
    assert D[p] == f32bits(2.0) and RG[p] == (10 << 32 | 20) and BA[p] == (30 << 32 | 1)
    assert np.count_nonzero(out) == 1
    # k points at one depth: floor of the per-channel mean.
    cols = [(255, 0, 7), (1, 2, 3), (100, 50, 25)]
    out, *_ = _hq_image(orc, make_points([(0, 0, 3.0)] * 3, [rgb(*c) for c in cols]), m, W, H)
    assert out[p] == rgb(356 // 3, 52 // 3, 35 // 3)
    # A point 0.5% behind the closest one blends in; one 2% behind does not.
    out, *_ = _hq_image(orc, make_points([(0, 0, 2.0), (0, 0, 2.01), (0, 0, 2.04)],
                                         [rgb(200, 100, 0), rgb(100, 0, 50), rgb(0, 255, 255)]),
                        m, W, H)
    assert out[p] == rgb(150, 50, 25)
    # The threshold is fl32(closest * 1.01f), inclusive.
    thr = np.float32(2.0) * np.float32(1.01)
    above = np.nextafter(thr, np.float32(np.inf), dtype=np.float32)
    out, *_ = _hq_image(orc, make_points([(0, 0, 2.0), (0, 0, float(thr))],
                                         [rgb(0, 0, 0), rgb(100, 100, 100)]), m, W, H)
    assert out[p] == rgb(50, 50, 50)
    out, *_ = _hq_image(orc, make_points([(0, 0, 2.0), (0, 0, float(above))],
                                         [rgb(0, 0, 0), rgb(100, 100, 100)]), m, W, H)
    assert out[p] == rgb(0, 0, 0)
    # The closest point always counts, in any arrival order.
    out, D, RG, BA = _hq_image(orc, make_points([(0, 0, 9.0), (0, 0, 1.0)], [rgb(9, 9, 9), rgb(1, 2, 3)]),
                               m, W, H)
    assert out[p] == rgb(1, 2, 3) and (int(BA[p]) & 0xFFFFFFFF) == 1


def check_resolve_hq(orc):
    RG = np.array([0, (7 << 32) | 9, (1000 << 32) | 255 * 4, 0], np.uint64)
    BA = np.array([0, (5 << 32) | 2, (4 << 32) | 4, 5 << 32], np.uint64)
    out = orc.resolve_hq(RG, BA, 2, 2)
    assert out.tolist() == [0, 3 | 4 << 8 | 2 << 16 | 0xFF000000,
                            (250 & 255) | 255 << 8 | 1 << 16 | 0xFF000000, 0]


def brute_force_hq(pid, dbits, rgba, W, H):
    """Per-pixel gather of the blend: closest depth, then the colour average
    over the points whose depth is within fl32(closest * 1.01f)."""
    out = np.zeros(W * H, np.uint32)
    for p in range(W * H):
        hit = np.nonzero(pid == p)[0]
        if len(hit) == 0:
            continue
        dmin = min(int(dbits[i]) for i in hit)
        thr = np.float32(bits2f(dmin)) * np.float32(1.01)
        sel = [i for i in hit if np.float32(bits2f(int(dbits[i]))) <= thr]
        s = [sum((int(rgba[i]) >> (8 * c)) & 255 for i in sel) for c in range(3)]
        k = len(sel)
        out[p] = (s[0] // k) | (s[1] // k) << 8 | (s[2] // k) << 16 | 255 << 24
    return out


def check_hq_brute_force(orc):
    for seed in range(2):
        pts, m, W, H = _dense_tiny_cloud(20 + seed)
        pid, d = orc.project_all(pts, m, W, H)
        out, *_ = _hq_image(orc, pts, m, W, H)
        assert np.array_equal(out, brute_force_hq(pid, d, pts["rgba"], W, H))


def check_hq_reduces_to_basic(orc):
    """When every point of a pixel is more than 1% behind the closest one,
    the blend shows exactly the closest point (= the basic image, alpha 255)."""
    W, H = 16, 16
    m = identity(m14=1.0, m15=0.0)
    rng = np.random.default_rng(5)
    xyz, cols = [], []
    for px in range(W):
        for py in range(H):
            X = (px + 0.5) / (W / 2) - 1
            Y = (py + 0.5) / (H / 2) - 1
            for k in range(int(rng.integers(0, 4))):
                z = 1.0 * (1.05 ** int(rng.integers(0, 30)))
                xyz.append((X * z, Y * z, z))
                cols.append(int(synth.pack_rgba(*rng.integers(0, 256, 3))))
    pts = make_points(xyz, cols)
    pid, d = orc.project_all(pts, m, W, H)
    # keep one point per (pixel, depth) so that ties cannot blend
    key = pid.astype(np.uint64) << 32 | d
    _, first = np.unique(key, return_index=True)
    pts = pts[np.sort(first)]
    out, *_ = _hq_image(orc, pts, m, W, H)
    basic = orc.resolve_basic(orc.render_basic(pts, m, W, H), W, H)
    assert np.array_equal(out, basic)


def check_hq_permutation(orc):
    pts, m, W, H = _dense_tiny_cloud(31)
    ref = _hq_image(orc, pts, m, W, H)
    rng = np.random.default_rng(9)
    perm = rng.permutation(len(pts))
    got = _hq_image(orc, pts[perm], m, W, H)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Vertex orders (Sec. 4, Sec. 5)
# ---------------------------------------------------------------------------

SPLITMIX_1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                    4593380528125082431, 16408922859458223821]


def check_splitmix64(orc):
    """Published SplitMix64 test vector: the first outputs for seed 1234567."""
    assert [orc.splitmix64(1234567, k) for k in range(5)] == SPLITMIX_1234567


def interleave_by_strings(qx, qy, qz):
    """Morton code built from binary digit strings (most significant first)."""
    bx, by, bz = (format(q, "021b") for q in (qx, qy, qz))
    return int("".join(z + y + x for x, y, z in zip(bx, by, bz)), 2)


def check_morton_interleave(orc):
    hand = {(1, 0, 0): 1, (0, 1, 0): 2, (0, 0, 1): 4, (1, 1, 1): 7, (2, 0, 0): 8,
            (0, 2, 0): 16, (3, 0, 0): 9, (2**21 - 1,) * 3: 2**63 - 1, (2**20, 0, 0): 1 << 60}
    for q, c in hand.items():
        assert orc.morton_interleave(*q) == c, (q, orc.morton_interleave(*q))
    rng = np.random.default_rng(1)
    for _ in range(300):
        q = [int(v) for v in rng.integers(0, 2**21, 3)]
        assert orc.morton_interleave(*q) == interleave_by_strings(*q)


def check_morton_quantisation(orc):
    """With the bounding cube [0, 2^21]^3 the cell index is the integer
    coordinate itself (the top face clamps to 2^21 - 1)."""
    rng = np.random.default_rng(2)
    q = rng.integers(0, 2**21, (500, 3))
    xyz = np.concatenate([q, [[0, 0, 0], [2**21, 5, 7], [3, 2**21, 2**21]]]).astype(np.float64)
    pts = make_points(xyz, np.zeros(len(xyz), np.uint32))
    codes = orc.morton_codes(pts)
    lo, hi = orc.bbox(pts)
    assert lo.tolist() == [0, 0, 0] and hi.tolist() == [2**21] * 3
    for i, (x, y, z) in enumerate(xyz.astype(np.int64)):
        c = [min(int(v), 2**21 - 1) for v in (x, y, z)]
        assert int(codes[i]) == interleave_by_strings(*c)
    # A flat cloud: the cube's edge is the longest extent, so y is quantised
    # against the x extent (y in [0, 1/4] -> at most 2^19).
    pts = make_points([(0, 0, 0), (4.0, 1.0, 0), (2.0, 0.5, 0)], [0, 0, 0])
    codes = orc.morton_codes(pts)
    assert int(codes[1]) == interleave_by_strings(2**21 - 1, 2**19, 0)
    assert int(codes[2]) == interleave_by_strings(2**20, 2**18, 0)
    # All points equal: every code is 0.
    pts = make_points([(1.5, 2.5, 3.5)] * 4, [0] * 4)
    assert orc.morton_codes(pts).tolist() == [0] * 4


def splitmix64_py(seed, k):
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & FULL
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & FULL
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & FULL
    return z ^ (z >> 31)


def check_reorder(orc, n=3000, batch=128, seed=17):
    rng = np.random.default_rng(4)
    xyz = rng.uniform(0, 10, (n, 3))
    xyz[n - 200:] = xyz[:200]                 # duplicated positions: equal codes
    pts = make_points(xyz, np.arange(n, dtype=np.uint32))
    codes = orc.morton_codes(pts)
    for order in (0, 1, 2):
        perm = orc.reorder(pts, order, batch, seed)
        assert np.array_equal(np.sort(perm), np.arange(n, dtype=np.uint32)), order
    mort = orc.reorder(pts, 0, batch, seed)
    c = codes[mort]
    assert np.all(c[1:] >= c[:-1])
    tie = c[1:] == c[:-1]
    assert tie.sum() >= 150 and np.all(mort[1:][tie] > mort[:-1][tie])      # stable
    # Shuffled Morton: runs of `batch` consecutive Morton positions, emitted in
    # the order of the batches' SplitMix64 keys.
    sm = orc.reorder(pts, 1, batch, seed)
    nb = (n + batch - 1) // batch
    keys = sorted(range(nb), key=lambda b: (splitmix64_py(seed, b), b))
    expect = np.concatenate([mort[b * batch:(b + 1) * batch] for b in keys])
    assert np.array_equal(sm, expect)
    assert not np.array_equal(sm, mort)
    # Shuffled: sort of the per-point keys.
    sh = orc.reorder(pts, 2, batch, seed)
    expect = sorted(range(n), key=lambda i: (splitmix64_py(seed, i), i))
    assert sh.tolist() == expect


def check_reorder_edges(orc):
    one = make_points([(1, 2, 3)], [5])
    for order in (0, 1, 2):
        assert orc.reorder(one, order).tolist() == [0]
        assert orc.reorder(one[:0], order).tolist() == []
    pts = make_points(np.random.default_rng(0).uniform(0, 1, (300, 3)), np.zeros(300, np.uint32))
    mort = orc.reorder(pts, 0)
    # batch = 1 shuffles single points of the Morton order; batch >= n is Morton.
    assert np.array_equal(orc.reorder(pts, 1, batch=300), mort)
    assert np.array_equal(orc.reorder(pts, 1, batch=1000), mort)
    b1 = orc.reorder(pts, 1, batch=1, seed=3)
    keys = sorted(range(300), key=lambda b: (splitmix64_py(3, b), b))
    assert np.array_equal(b1, mort[keys])


def check_image_order_invariance(orc):
    """The rendered image does not depend on the vertex order (Sec. 4 only
    changes speed)."""
    pts, m, W, H = _dense_tiny_cloud(40, n=2000)
    ref = orc.render_basic(pts, m, W, H)
    refq = _hq_image(orc, pts, m, W, H)[0]
    for order in (0, 1, 2):
        perm = orc.reorder(pts, order, 128, 5)
        assert np.array_equal(orc.render_basic(pts[perm], m, W, H), ref)
        assert np.array_equal(_hq_image(orc, pts[perm], m, W, H)[0], refq)


def check_golden_scene(orc):
    """A small scene whose images and orders were written by
    tests/golden/make_golden.py (oracle only) when the pins above passed."""
    with open(os.path.join(GOLDEN, "tiny_scene.json")) as f:
        g = json.load(f)
    pts = synth.buildings(g["n"], seed=g["seed"])
    m = np.array(g["mvp"], np.float32)
    W, H = g["W"], g["H"]
    fb = orc.render_basic(pts, m, W, H)
    out = orc.resolve_basic(fb, W, H)
    hq, *_ = _hq_image(orc, pts, m, W, H)
    import hashlib
    assert hashlib.sha256(out.tobytes()).hexdigest() == g["basic_sha256"]
    assert hashlib.sha256(hq.tobytes()).hexdigest() == g["hq_sha256"]
    perm = orc.reorder(pts, 1, 128, g["seed"])
    assert hashlib.sha256(perm.tobytes()).hexdigest() == g["morton_shuffle_sha256"]


# ---------------------------------------------------------------------------
# Depth output of the resolve (Sec. 3.1, closing paragraph)
# ---------------------------------------------------------------------------

def gl_perspective64(fovy_deg, aspect, near, far):
    """The usual OpenGL projection matrix, float64, row-major."""
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2)
    return np.array([[f / aspect, 0, 0, 0], [0, f, 0, 0],
                     [0, 0, (far + near) / (near - far), 2 * far * near / (near - far)],
                     [0, 0, -1, 0]], np.float64)


def window_depth64(P, w):
    """Window depth in [0,1] that the fixed-function pipeline derives from
    clip z / clip w for view-space points at distance w in front of the camera."""
    v = np.stack([np.zeros_like(w), np.zeros_like(w), -w, np.ones_like(w)])
    c = P @ v
    return (c[2] / c[3] + 1.0) / 2.0


def check_depth_linear(orc):
    """The linear depth of a pixel is the w of its closest point; uncovered
    pixels get the caller's value (hand case: w = z, pixel centres)."""
    W, H = 4, 4
    m = identity(m14=1.0, m15=0.0)
    cells = {(0, 0): [3.0, 1.5, 2.0], (3, 1): [0.25], (2, 3): [7.0, 7.5]}
    xyz, cols = [], []
    for (px, py), zs in cells.items():
        X, Y = (px + 0.5) / (W / 2) - 1, (py + 0.5) / (H / 2) - 1
        for z in zs:
            xyz.append((X * z, Y * z, z))
            cols.append(0x11223344)
    pts = make_points(xyz, cols)
    fb = orc.render_basic(pts, m, W, H)
    out = orc.resolve_depth_basic(fb, W, H, 0, 0.0, 0.0, -1.0)
    want = np.full(W * H, -1.0, np.float32)
    for (px, py), zs in cells.items():
        want[py * W + px] = min(zs)
    assert np.array_equal(out, want), out
    D, _, _ = orc.render_hq(pts, m, W, H)
    assert np.array_equal(orc.resolve_depth_hq(D, W, H, 0, 0.0, 0.0, -1.0), want)


def check_depth_window(orc):
    """With a = f/(f-n), b = -f*n/(f-n) the hyperbolic depth is the window
    depth of an OpenGL perspective projection (float64 through the matrix),
    within the rounding bound of three float32 operations and two rounded
    coefficients; with the reverse-z coefficients it is one minus that.
    Both are monotone in w, and the near and far planes map to 0 and 1."""
    u = 2.0 ** -24
    rng = np.random.default_rng(21)
    for near, far in ((0.1, 1000.0), (1.0, 100.0), (0.5, 5e4)):
        P = gl_perspective64(60.0, 16 / 9, near, far)
        w = np.sort(np.concatenate([[near, far], near * (far / near) ** rng.random(2000)]))
        w = w.astype(np.float32)
        fb = (w.view(np.uint32).astype(np.uint64) << np.uint64(32)) | np.uint64(0xFF00FF00)
        n = len(w)
        w64 = w.astype(np.float64)
        exact = window_depth64(P, w64)
        for reverse in (False, True):
            a64 = -near / (far - near) if reverse else far / (far - near)
            b64 = far * near / (far - near) * (1 if reverse else -1)
            a, b = float(np.float32(a64)), float(np.float32(b64))
            got = orc.resolve_depth_basic(fb, n, 1, 1, a, b, -1.0).astype(np.float64)
            want = 1.0 - exact if reverse else exact
            bound = 2 * u * (abs(a64) + 2 * np.abs(b64 / w64) + np.abs(want)) + 1e-12
            assert np.all(np.abs(got - want) <= bound), (near, far, reverse, np.max(np.abs(got - want) - bound))
            d = np.diff(got)
            assert np.all(d <= 0) if reverse else np.all(d >= 0)
            # the planes themselves, after rounding near and far to float32
            tol = 8 * u * (abs(a64) + abs(b64) / near)
            assert abs(got[0] - (1.0 if reverse else 0.0)) <= tol, (near, far, reverse, got[0])
            assert abs(got[-1] - (0.0 if reverse else 1.0)) <= tol, (near, far, reverse, got[-1])


def check_depth_dyadic(orc):
    """Dyadic coefficients and depths: every step is exact."""
    w = np.array([0.5, 0.25, 2.0, 1.0, 8.0], np.float32)
    fb = (w.view(np.uint32).astype(np.uint64) << np.uint64(32)) | np.uint64(7)
    fb = np.concatenate([fb, [np.uint64(FULL)]])
    got = orc.resolve_depth_basic(fb, 6, 1, 1, 0.5, -0.25, 3.0)
    assert got.tolist() == [0.0, -0.5, 0.375, 0.25, 0.46875, 3.0], got


def check_depth_hq_equals_basic(orc):
    """The HQ depth pass keeps the same closest depth as the basic key, so
    both depth images agree in every mode."""
    pts, m, W, H = _dense_tiny_cloud(23)
    fb = orc.render_basic(pts, m, W, H)
    D, _, _ = orc.render_hq(pts, m, W, H)
    for mode, a, b in ((0, 0.0, 0.0), (1, 1.0009995, -0.10004998)):
        x = orc.resolve_depth_basic(fb, W, H, mode, a, b, -2.0)
        y = orc.resolve_depth_hq(D, W, H, mode, a, b, -2.0)
        assert np.array_equal(x, y)
        assert np.any(x == -2.0) and np.any(x != -2.0)


# ---------------------------------------------------------------------------
# Single-atomic HQ form (Sec. 3.5.1: 18-bit colour sums and a 10-bit count in
# one 64-bit word; field order r, g, b, count from the top is this project's
# reading)
# ---------------------------------------------------------------------------

def _packed(r, g, b):
    return (r << 46) | (g << 28) | (b << 10) | 1


def _resolve_packed_by_hand(word):
    a = word & 0x3FF
    if a == 0:
        return 0
    r, g, b = (word >> 46) & 0x3FFFF, (word >> 28) & 0x3FFFF, (word >> 10) & 0x3FFFF
    return (r // a & 255) | (g // a & 255) << 8 | (b // a & 255) << 16 | 0xFF000000


def check_hq_packed_matches_two_words(orc):
    """With at most 1023 points per pixel the packed word holds exactly the
    two-word sums (count, red, green, blue) and resolves to the same image."""
    rng = np.random.default_rng(31)
    W, H = 48, 32
    m = synth.mvp((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), W, H, fovy=50.0)
    xyz = rng.uniform(-1.6, 1.6, (30_000, 3))
    xyz[10_000:20_000] = xyz[:10_000]                   # equal depths: several points blend
    pts = make_points(xyz, rng.integers(0, 2**32, len(xyz), dtype=np.uint64).astype(np.uint32))
    D, RG, BA = orc.render_hq(pts, m, W, H)
    D2, P = orc.render_hq_packed(pts, m, W, H)
    assert np.array_equal(D, D2)
    cnt = BA & np.uint64(0xFFFFFFFF)
    assert int(cnt.max()) <= 1023 and int(cnt.max()) >= 2
    assert np.array_equal(P & np.uint64(0x3FF), cnt)
    assert np.array_equal((P >> np.uint64(46)) & np.uint64(0x3FFFF), RG >> np.uint64(32))
    assert np.array_equal((P >> np.uint64(28)) & np.uint64(0x3FFFF), RG & np.uint64(0xFFFFFFFF))
    assert np.array_equal((P >> np.uint64(10)) & np.uint64(0x3FFFF), BA >> np.uint64(32))
    assert np.array_equal(orc.resolve_hq_packed(P, W, H), orc.resolve_hq(RG, BA, W, H))


def check_hq_packed_overflow(orc):
    """Points at one pixel and one depth: the packed word is the sum of the
    per-point packed values modulo 2^64 (computed here with Python integers),
    and the resolve follows by hand.  1023 points are exact; 1024 wrap the
    count to 0 (the pixel resolves empty, the paper's artifact); 1025 carry
    one into the blue field."""
    W, H = 8, 8
    m = identity(m14=1.0, m15=0.0)   # clip w = z, pixel (4,4) for x = y = 0
    p = 4 * W + 4
    rng = np.random.default_rng(32)
    for k in (1, 2, 1023, 1024, 1025, 2100):
        cols = rng.integers(0, 256, (k, 3))
        cols[: k // 2] = 255                              # drive the fields towards their width
        rgba = [int(synth.pack_rgba(int(r), int(g), int(b))) for r, g, b in cols]
        D, P = orc.render_hq_packed(make_points([(0, 0, 2.0)] * k, rgba), m, W, H)
        want = sum(_packed(int(r), int(g), int(b)) for r, g, b in cols) % (1 << 64)
        assert int(P[p]) == want, (k, hex(int(P[p])), hex(want))
        assert np.count_nonzero(P) == 1
        img = orc.resolve_hq_packed(P, W, H)
        assert int(img[p]) == _resolve_packed_by_hand(want), k
        if k <= 1023:
            sums = cols.sum(axis=0)
            assert int(img[p]) == int(synth.pack_rgba(*(int(x) // k for x in sums)))
        if k == 1024:
            assert int(img[p]) == 0
    # The threshold is inclusive here too: a point exactly at fl32(closest *
    # 1.01f) counts, the next float above does not.
    thr = np.float32(2.0) * np.float32(1.01)
    above = np.nextafter(thr, np.float32(np.inf), dtype=np.float32)
    for z, count in ((float(thr), 2), (float(above), 1)):
        _, P = orc.render_hq_packed(make_points([(0, 0, 2.0), (0, 0, z)], [0, 0]), m, W, H)
        assert int(P[p]) & 0x3FF == count, (z, int(P[p]))


def check_resolve_hq_packed(orc):
    words = [0, _packed(9, 18, 27), _packed(255, 0, 7) + _packed(1, 2, 3) + _packed(100, 50, 25),
             (5 << 46) | (6 << 28) | (7 << 10)]          # sums without a count: empty
    out = orc.resolve_hq_packed(np.array(words, np.uint64), 2, 2)
    assert out.tolist() == [0, 9 | 18 << 8 | 27 << 16 | 0xFF000000,
                            (356 // 3) | (52 // 3) << 8 | (35 // 3) << 16 | 0xFF000000, 0]


ALL_CHECKS = [
    check_hand_cases, check_projection_fp64, check_projection_dyadic, check_projection_rounding,
    check_basic_brute_force, check_basic_permutation, check_basic_accumulate,
    check_basic_closest_wins, check_resolve_basic,
    check_hq_special_cases, check_resolve_hq, check_hq_brute_force, check_hq_reduces_to_basic,
    check_hq_permutation,
    check_splitmix64, check_morton_interleave, check_morton_quantisation, check_reorder,
    check_reorder_edges, check_image_order_invariance,
    check_depth_linear, check_depth_window, check_depth_dyadic, check_depth_hq_equals_basic,
    check_hq_packed_matches_two_words, check_hq_packed_overflow, check_resolve_hq_packed,
]
