"""CPU oracle for the compute point rasterizer (ctypes wrapper over pcr_oracle.c).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark load this module; the library under test never imports it and
shares no code with it.

Every function here follows the C oracle one to one; the C file names the
paper passage each step follows (Sec. 3.1 basic render and resolve, Sec. 3.5 HQ
depth/colour/resolve, Sec. 4 and Sec. 5 vertex orders).

Points are any C-contiguous array of 16-byte records {f32 x, y, z; u32 rgba}
(for instance ``paper_2104_07526_amd.synth.POINT_DTYPE``); the matrix is 16
float32 values, row-major.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libpcr_oracle.so")

# One rounding per float operation, no contraction into FMA, no fast-math, SSE
# arithmetic (no x87 excess precision).
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-msse2", "-mfpmath=sse", "-fexcess-precision=standard"]

_lock = threading.Lock()
_lib = None

ORDER_MORTON = 0
ORDER_MORTON_SHUFFLE = 1
ORDER_SHUFFLE = 2


def build(out_path: str = _LIB_PATH, extra_flags=()) -> str:
    """Compiles the oracle with gcc into ``out_path`` and returns the path."""
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", out_path, _SRC]
    subprocess.run(cmd, check=True)
    return out_path


def _declare(lib):
    P = ctypes.c_void_p
    U32, U64, I32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    F = ctypes.c_float
    sig = {
        "oracle_fp_env_ok": (I32, []),
        "oracle_project": (I32, [P, U32, U32, F, F, F, P, P]),
        "oracle_project_all": (None, [P, U64, P, U32, U32, P, P]),
        "oracle_clear_basic": (None, [P, U32, U32]),
        "oracle_render_basic": (None, [P, U64, P, U32, U32, P]),
        "oracle_resolve_basic": (None, [P, U32, U32, P]),
        "oracle_clear_hq": (None, [P, P, P, U32, U32]),
        "oracle_render_hq_depth": (None, [P, U64, P, U32, U32, P]),
        "oracle_render_hq_color": (None, [P, U64, P, U32, U32, P, P, P]),
        "oracle_render_hq": (None, [P, U64, P, U32, U32, P, P, P]),
        "oracle_resolve_hq": (None, [P, P, U32, U32, P]),
        "oracle_render_hq_packed_color": (None, [P, U64, P, U32, U32, P, P]),
        "oracle_resolve_hq_packed": (None, [P, U32, U32, P]),
        "oracle_resolve_depth_basic": (None, [P, U32, U32, I32, F, F, F, P]),
        "oracle_resolve_depth_hq": (None, [P, U32, U32, I32, F, F, F, P]),
        "oracle_splitmix64": (U64, [U64, U64]),
        "oracle_bbox": (None, [P, U64, P, P]),
        "oracle_morton_interleave": (U64, [U32, U32, U32]),
        "oracle_morton_codes": (None, [P, U64, P]),
        "oracle_reorder": (I32, [P, U64, I32, U32, U64, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load(path: str | None = None):
    """Loads the oracle library (building it first if it is not built).

    With ``path`` given, loads that build (used by the mutation tests) without
    caching it."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def _pts(points):
    a = np.ascontiguousarray(points)
    rec = a.dtype.itemsize * (a.shape[1] if a.ndim == 2 else 1)
    if a.ndim not in (1, 2) or rec != 16:
        raise ValueError("points must be an array of 16-byte records")
    return a


def _n(points):
    return np.asarray(points).shape[0]


def _mvp(m):
    m = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(16))
    return m


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Thin object form so that a test can bind a different build (mutants)."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # -- projection -------------------------------------------------------
    def fp_env_ok(self) -> bool:
        return bool(self.lib.oracle_fp_env_ok())

    def project(self, m, W, H, x, y, z):
        """(pid, depth_bits) of one point, or None when culled."""
        m = _mvp(m)
        pid = ctypes.c_uint32()
        d = ctypes.c_uint32()
        ok = self.lib.oracle_project(_ptr(m), W, H, float(np.float32(x)),
                                     float(np.float32(y)), float(np.float32(z)),
                                     ctypes.byref(pid), ctypes.byref(d))
        return (pid.value, d.value) if ok else None

    def project_all(self, points, m, W, H):
        """Arrays (pid, depth_bits); culled points get 0xFFFFFFFF in both."""
        p = _pts(points)
        n = _n(p)
        m = _mvp(m)
        pid = np.empty(n, np.uint32)
        d = np.empty(n, np.uint32)
        self.lib.oracle_project_all(_ptr(p), n, _ptr(m), W, H, _ptr(pid), _ptr(d))
        return pid, d

    # -- basic --------------------------------------------------------------
    def clear_basic(self, W, H):
        fb = np.empty(W * H, np.uint64)
        self.lib.oracle_clear_basic(_ptr(fb), W, H)
        return fb

    def render_basic(self, points, m, W, H, fb=None):
        """Key framebuffer (u64[W*H]); accumulates into ``fb`` when given."""
        if fb is None:
            fb = self.clear_basic(W, H)
        p = _pts(points)
        m = _mvp(m)
        self.lib.oracle_render_basic(_ptr(p), _n(p), _ptr(m), W, H, _ptr(fb))
        return fb

    def resolve_basic(self, fb, W, H):
        fb = np.ascontiguousarray(fb, dtype=np.uint64)
        out = np.empty(W * H, np.uint32)
        self.lib.oracle_resolve_basic(_ptr(fb), W, H, _ptr(out))
        return out

    # -- HQ -----------------------------------------------------------------
    def clear_hq(self, W, H):
        D = np.empty(W * H, np.uint32)
        RG = np.empty(W * H, np.uint64)
        BA = np.empty(W * H, np.uint64)
        self.lib.oracle_clear_hq(_ptr(D), _ptr(RG), _ptr(BA), W, H)
        return D, RG, BA

    def render_hq(self, points, m, W, H, bufs=None, passes="both"):
        """(D, RG, BA) after the depth and/or colour pass."""
        D, RG, BA = bufs if bufs is not None else self.clear_hq(W, H)
        p = _pts(points)
        m = _mvp(m)
        n = _n(p)
        if passes in ("both", "depth"):
            self.lib.oracle_render_hq_depth(_ptr(p), n, _ptr(m), W, H, _ptr(D))
        if passes in ("both", "color"):
            self.lib.oracle_render_hq_color(_ptr(p), n, _ptr(m), W, H, _ptr(D),
                                            _ptr(RG), _ptr(BA))
        return D, RG, BA

    def resolve_hq(self, RG, BA, W, H):
        RG = np.ascontiguousarray(RG, dtype=np.uint64)
        BA = np.ascontiguousarray(BA, dtype=np.uint64)
        out = np.empty(W * H, np.uint32)
        self.lib.oracle_resolve_hq(_ptr(RG), _ptr(BA), W, H, _ptr(out))
        return out

    def render_hq_packed(self, points, m, W, H, D=None, P=None, passes="both"):
        """(D, P) of the single-atomic HQ form: the depth pass as render_hq,
        then one packed 18-18-18-10 word per pixel (Sec. 3.5.1)."""
        if D is None:
            D = np.full(W * H, 0xFFFFFFFF, np.uint32)
        if P is None:
            P = np.zeros(W * H, np.uint64)
        p = _pts(points)
        m = _mvp(m)
        n = _n(p)
        if passes in ("both", "depth"):
            self.lib.oracle_render_hq_depth(_ptr(p), n, _ptr(m), W, H, _ptr(D))
        if passes in ("both", "color"):
            self.lib.oracle_render_hq_packed_color(_ptr(p), n, _ptr(m), W, H, _ptr(D), _ptr(P))
        return D, P

    def resolve_hq_packed(self, P, W, H):
        P = np.ascontiguousarray(P, dtype=np.uint64)
        out = np.empty(W * H, np.uint32)
        self.lib.oracle_resolve_hq_packed(_ptr(P), W, H, _ptr(out))
        return out

    def resolve_depth_basic(self, fb, W, H, mode=0, a=0.0, b=0.0, empty=float("inf")):
        """Depth image (float32[W*H]) of a basic framebuffer: w, or a + b/w."""
        fb = np.ascontiguousarray(fb, dtype=np.uint64)
        out = np.empty(W * H, np.float32)
        self.lib.oracle_resolve_depth_basic(_ptr(fb), W, H, mode, a, b, empty, _ptr(out))
        return out

    def resolve_depth_hq(self, D, W, H, mode=0, a=0.0, b=0.0, empty=float("inf")):
        """Depth image (float32[W*H]) of an HQ depth buffer: w, or a + b/w."""
        D = np.ascontiguousarray(D, dtype=np.uint32)
        out = np.empty(W * H, np.float32)
        self.lib.oracle_resolve_depth_hq(_ptr(D), W, H, mode, a, b, empty, _ptr(out))
        return out

    # -- orders ---------------------------------------------------------------
    def splitmix64(self, seed, k):
        return int(self.lib.oracle_splitmix64(seed, k))

    def bbox(self, points):
        p = _pts(points)
        lo = np.zeros(3, np.float32)
        hi = np.zeros(3, np.float32)
        self.lib.oracle_bbox(_ptr(p), _n(p), _ptr(lo), _ptr(hi))
        return lo, hi

    def morton_interleave(self, qx, qy, qz):
        return int(self.lib.oracle_morton_interleave(qx, qy, qz))

    def morton_codes(self, points):
        p = _pts(points)
        out = np.empty(_n(p), np.uint64)
        self.lib.oracle_morton_codes(_ptr(p), _n(p), _ptr(out))
        return out

    def reorder(self, points, order, batch=128, seed=0):
        """perm (u32[n]): perm[j] is the input index of output point j."""
        p = _pts(points)
        n = _n(p)
        perm = np.empty(n, np.uint32)
        rc = self.lib.oracle_reorder(_ptr(p), n, order, batch, seed, _ptr(perm))
        if rc != 0:
            raise ValueError("oracle_reorder rejected its arguments")
        return perm


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
