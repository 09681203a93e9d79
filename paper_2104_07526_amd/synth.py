"""Seeded synthetic point clouds and cameras.

This module holds no step of the rendering method: it only produces inputs
(16-byte points and a float32 row-major model-view-projection matrix), the same
for the GPU library and for the CPU oracle.  The shapes stand in for the scans
the paper measures on (Sec. 5: a terrestrial town scan, a building site, small
statues), which are not available here.

All geometry is computed in float64 and rounded to float32 once.  Large clouds
are generated in fixed chunks of ``CHUNK`` points, each with its own
``numpy.random.Generator`` keyed by (seed, chunk index), so the result does not
depend on the number of worker threads.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

POINT_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("rgba", "<u4")])
CHUNK = 1 << 22

_TERRAIN_STOPS = np.array([[34, 85, 34], [107, 142, 35], [139, 115, 85], [240, 240, 240]],
                          dtype=np.float64)


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def empty_points(n: int, out=None) -> np.ndarray:
    if out is None:
        return np.empty(n, POINT_DTYPE)
    if out.dtype != POINT_DTYPE or out.shape != (n,):
        raise ValueError("out must be a POINT_DTYPE array of length n")
    return out


def pack_rgba(r, g, b, a=255):
    r = np.asarray(r, np.uint32)
    g = np.asarray(g, np.uint32)
    b = np.asarray(b, np.uint32)
    a = np.asarray(a, np.uint32)
    return (r & 255) | ((g & 255) << 8) | ((b & 255) << 16) | ((a & 255) << 24)


def _chunked(n, fill, seed, out):
    """Calls fill(rng, start, stop, view) for each chunk, in parallel."""
    pts = empty_points(n, out)
    nchunks = (n + CHUNK - 1) // CHUNK

    def run(c):
        s = c * CHUNK
        e = min(n, s + CHUNK)
        rng = np.random.default_rng([seed, c])
        fill(rng, s, e, pts[s:e])

    if nchunks <= 1:
        for c in range(nchunks):
            run(c)
    else:
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(run, range(nchunks)))
    return pts


# ---------------------------------------------------------------------------
# Clouds
# ---------------------------------------------------------------------------

def sphere(n: int, seed: int = 1, out=None) -> np.ndarray:
    """Points uniform on the unit sphere (normalised N(0, I3)), uniformly random
    RGBA bytes; the generation order is a random order."""

    def fill(rng, s, e, v):
        g = rng.standard_normal((e - s, 3))
        g /= np.linalg.norm(g, axis=1, keepdims=True)
        v["x"] = g[:, 0]
        v["y"] = g[:, 1]
        v["z"] = g[:, 2]
        v["rgba"] = rng.integers(0, 1 << 32, size=e - s, dtype=np.uint64).astype(np.uint32)

    return _chunked(n, fill, seed, out)


class TerrainParams:
    """Sum of eight random sines over a square area (a LiDAR-like heightfield)."""

    def __init__(self, seed: int, extent: float = 1000.0, waves: int = 8):
        rng = np.random.default_rng([seed, 0x7E55A1])
        self.extent = float(extent)
        self.amp = rng.uniform(1.0, 20.0, waves)
        self.wavelength = rng.uniform(30.0, 600.0, waves)
        ang = rng.uniform(0.0, 2.0 * math.pi, waves)
        self.dir = np.stack([np.cos(ang), np.sin(ang)], axis=1)
        self.phase = rng.uniform(0.0, 2.0 * math.pi, waves)
        self.zspan = float(self.amp.sum())

    def height(self, x, y):
        z = np.zeros_like(x)
        for k in range(len(self.amp)):
            t = (self.dir[k, 0] * x + self.dir[k, 1] * y) * (2.0 * math.pi / self.wavelength[k])
            z += self.amp[k] * np.sin(t + self.phase[k])
        return z


def _ramp(t):
    t = np.clip(t, 0.0, 1.0) * (len(_TERRAIN_STOPS) - 1)
    i = np.minimum(t.astype(np.int64), len(_TERRAIN_STOPS) - 2)
    f = (t - i)[:, None]
    c = _TERRAIN_STOPS[i] * (1.0 - f) + _TERRAIN_STOPS[i + 1] * f
    return np.rint(c).astype(np.uint32)


def terrain(n: int, seed: int = 2, extent: float = 1000.0, out=None) -> np.ndarray:
    """Jittered-grid heightfield over extent x extent metres in scanline order
    (row-major over the grid, the order a line scanner would emit)."""
    prm = TerrainParams(seed, extent)
    side = max(1, math.isqrt(n))
    if side * side < n:
        side += 1
    spacing = extent / side

    def fill(rng, s, e, v):
        idx = np.arange(s, e, dtype=np.int64)
        row = idx // side
        col = idx - row * side
        jit = rng.random((e - s, 2))
        x = (col + jit[:, 0]) * spacing
        y = (row + jit[:, 1]) * spacing
        z = prm.height(x, y) + rng.normal(0.0, 0.01, e - s)
        rgb = _ramp((z + prm.zspan) / (2.0 * prm.zspan))
        v["x"] = x
        v["y"] = y
        v["z"] = z
        v["rgba"] = pack_rgba(rgb[:, 0], rgb[:, 1], rgb[:, 2])

    return _chunked(n, fill, seed, out)


class BuildingLayout:
    """A ground square plus random axis-aligned boxes (four walls and a roof),
    added until the total surface reaches ``area`` square metres."""

    def __init__(self, seed: int, ground: float = 250.0, area: float = 150_000.0,
                 origin=(375.0, 375.0)):
        rng = np.random.default_rng([seed, 0xB0C5])
        ox, oy = origin
        # Each face: origin o, edge vectors a and b (point = o + u*a + v*b),
        # base colour, and a flag for the striped ground.
        faces = [((ox, oy, 0.0), (ground, 0, 0), (0, ground, 0), (128, 128, 128), True)]
        total = ground * ground
        while total < area:
            w, d = rng.uniform(10.0, 40.0, 2)
            h = rng.uniform(5.0, 60.0)
            x0 = ox + rng.uniform(0.0, ground - w)
            y0 = oy + rng.uniform(0.0, ground - d)
            cols = rng.integers(40, 216, size=(5, 3))
            box = [
                ((x0, y0, h), (w, 0, 0), (0, d, 0)),          # roof
                ((x0, y0, 0.0), (w, 0, 0), (0, 0, h)),        # south wall
                ((x0, y0 + d, 0.0), (w, 0, 0), (0, 0, h)),    # north wall
                ((x0, y0, 0.0), (0, d, 0), (0, 0, h)),        # west wall
                ((x0 + w, y0, 0.0), (0, d, 0), (0, 0, h)),    # east wall
            ]
            for (o, a, b), c in zip(box, cols):
                faces.append((o, a, b, tuple(int(t) for t in c), False))
                total += float(np.linalg.norm(np.cross(a, b)))
        self.faces = faces
        self.area = np.array([float(np.linalg.norm(np.cross(f[1], f[2]))) for f in faces])
        self.origin = np.array(origin, np.float64)
        self.ground = ground
        self.height = max(f[0][2] for f in faces[1:]) if len(faces) > 1 else 0.0

    def counts(self, n: int) -> np.ndarray:
        """Points per face, proportional to area, summing to exactly n."""
        share = self.area / self.area.sum() * n
        c = np.floor(share).astype(np.int64)
        rest = n - int(c.sum())
        if rest > 0:
            order = np.argsort(-(share - c), kind="stable")
            c[order[:rest]] += 1
        return c


def buildings(n: int, seed: int = 4, out=None) -> np.ndarray:
    """Building-scan-like scene, face by face (uniform density per face), colour
    = per-face base colour + per-point noise in [-24, 24]; the ground carries
    0.5 m stripes."""
    lay = BuildingLayout(seed)
    cnt = lay.counts(n)
    start = np.concatenate([[0], np.cumsum(cnt)])
    F = len(lay.faces)
    O = np.array([f[0] for f in lay.faces], np.float64)
    A = np.array([f[1] for f in lay.faces], np.float64)
    B = np.array([f[2] for f in lay.faces], np.float64)
    C = np.array([f[3] for f in lay.faces], np.int64)
    ground = np.array([f[4] for f in lay.faces])

    def fill(rng, s, e, v):
        idx = np.arange(s, e, dtype=np.int64)
        face = np.searchsorted(start, idx, side="right") - 1
        face = np.minimum(face, F - 1)
        uv = rng.random((e - s, 2))
        p = O[face] + uv[:, :1] * A[face] + uv[:, 1:] * B[face]
        col = C[face].copy()
        g = ground[face]
        if g.any():
            stripe = (np.floor(p[g, 0] / 0.5).astype(np.int64) & 1) == 1
            col[g] = np.where(stripe[:, None], [200, 190, 170], [90, 90, 95])
        col += rng.integers(-24, 25, size=(e - s, 3))
        col = np.clip(col, 0, 255)
        v["x"] = p[:, 0]
        v["y"] = p[:, 1]
        v["z"] = p[:, 2]
        v["rgba"] = pack_rgba(col[:, 0], col[:, 1], col[:, 2])

    return _chunked(n, fill, seed, out)


def terrain_and_buildings(n_terrain: int, n_build: int, seed: int = 5, out=None) -> np.ndarray:
    """Concatenation of a terrain cloud and a building cloud (one buffer)."""
    pts = empty_points(n_terrain + n_build, out)
    terrain(n_terrain, seed=seed, out=pts[:n_terrain])
    buildings(n_build, seed=seed + 1000, out=pts[n_terrain:])
    return pts


# ---------------------------------------------------------------------------
# Cameras (inputs: built in float64, rounded once to float32, row-major)
# ---------------------------------------------------------------------------

def look_at(eye, target, up) -> np.ndarray:
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, np.asarray(up, np.float64))
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    V = np.eye(4)
    V[0, :3], V[1, :3], V[2, :3] = s, u, -f
    V[0, 3], V[1, 3], V[2, 3] = -s @ eye, -u @ eye, f @ eye
    return V


def perspective(fovy_deg: float, aspect: float, near: float, far: float) -> np.ndarray:
    t = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    P = np.zeros((4, 4))
    P[0, 0] = t / aspect
    P[1, 1] = t
    P[2, 2] = (far + near) / (near - far)
    P[2, 3] = 2.0 * far * near / (near - far)
    P[3, 2] = -1.0
    return P


def mvp(eye, target, up, width: int, height: int, fovy: float = 60.0,
        near: float = 0.1, far: float = 10_000.0) -> np.ndarray:
    """Row-major float32[16]; clip w equals the distance along the view axis."""
    M = perspective(fovy, width / height, near, far) @ look_at(eye, target, up)
    return M.astype(np.float32).reshape(16)


def random_poses(count: int, seed: int = 5, center=(500.0, 500.0)):
    """Eyes on an annulus of radius 100-700 m around ``center`` at 30-400 m
    altitude, targets uniform in the central 500 m square on the ground."""
    rng = np.random.default_rng([seed, 0x905E])
    cx, cy = center
    poses = []
    for _ in range(count):
        r = rng.uniform(100.0, 700.0)
        a = rng.uniform(0.0, 2.0 * math.pi)
        eye = (cx + r * math.cos(a), cy + r * math.sin(a), rng.uniform(30.0, 400.0))
        tgt = (cx + rng.uniform(-250.0, 250.0), cy + rng.uniform(-250.0, 250.0), 0.0)
        poses.append((eye, tgt, (0.0, 0.0, 1.0)))
    return poses


# ---------------------------------------------------------------------------
# The workloads (resolution, cloud, camera) of the measured configurations
# ---------------------------------------------------------------------------

RESOLUTIONS = {"720p": (1280, 720), "1080p": (1920, 1080), "1440p": (2560, 1440),
               "4k": (3840, 2160)}


def sphere_view(width=1280, height=720):
    """Camera 3 units from the origin looking at it, 60 degree field of view."""
    return mvp((0.0, 0.0, 3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), width, height,
               near=0.1, far=10.0)


def terrain_oblique(width=1920, height=1080):
    """200 m altitude, 45 degree oblique view over the terrain."""
    return mvp((500.0, 300.0, 200.0), (500.0, 500.0, 0.0), (0.0, 0.0, 1.0), width, height)


def terrain_away(width=1920, height=1080):
    """Looking up into the sky: no point in the frustum (pure streaming)."""
    return mvp((500.0, 500.0, 500.0), (500.0, 500.0, 1000.0), (0.0, 1.0, 0.0), width, height)


def terrain_closeup(width=1920, height=1080):
    return mvp((500.0, 480.0, 25.0), (500.0, 520.0, 0.0), (0.0, 0.0, 1.0), width, height)


def terrain_overview(width=1920, height=1080):
    """Far away: the whole kilometre falls into a small part of the image."""
    return mvp((500.0, -6000.0, 4000.0), (500.0, 500.0, 0.0), (0.0, 0.0, 1.0), width, height,
               far=50_000.0)


def buildings_overview(width=2560, height=1440, seed=4):
    """From outside the bounding box at 45 degrees elevation, scene in view."""
    lay = BuildingLayout(seed)
    c = lay.origin + lay.ground / 2.0
    radius = 0.5 * math.sqrt(2.0 * lay.ground ** 2 + lay.height ** 2)
    dist = 1.15 * radius / math.tan(math.radians(30.0))
    e = math.radians(45.0)
    eye = (c[0] + dist * math.cos(e) * math.cos(-0.7), c[1] + dist * math.cos(e) * math.sin(-0.7),
           dist * math.sin(e))
    return mvp(eye, (c[0], c[1], 0.0), (0.0, 0.0, 1.0), width, height)
