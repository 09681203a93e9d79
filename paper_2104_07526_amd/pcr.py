"""ctypes binding of libpcr (include/pcr.h).  Argument marshalling only: every
step of rendering and reordering runs in the library's HIP kernels.

Buffers are torch tensors on the GPU (any dtype; only their bytes and device
pointers are used).  Work is enqueued on the current torch stream unless a
``stream`` (torch.cuda.Stream or raw handle) is given.  Nothing here
synchronises.

The library must be built (``python -m paper_2104_07526_amd.build``); loading
fails loudly otherwise, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcr.so")

BASIC, DEDUP, HQ = 0, 1, 2
F_EARLYZ = 1 << 8
F_REDUCE = 1 << 9
F_LDS = 1 << 10
F_PLAIN = 1 << 11
F_HQ_DEPTH = 1 << 12
F_HQ_COLOR = 1 << 13
F_HQ_PACKED = 1 << 14
F_HQ_ROBUST = 1 << 15
F_REDUCE_WAVE = 1 << 16
F_REDUCE_PAIR = 1 << 17
ORDER_MORTON, ORDER_MORTON_SHUFFLE, ORDER_SHUFFLE = 0, 1, 2
DEPTH_LINEAR, DEPTH_HYPERBOLIC = 0, 1

OK, EINVAL, EHIP, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -4

_lock = threading.Lock()
_lib = None


class PcrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pcr error {code}: {msg}")
        self.code = code


class Tune(ctypes.Structure):
    _fields_ = [("ppt", ctypes.c_uint32), ("wg", ctypes.c_uint32), ("grid", ctypes.c_uint32),
                ("group", ctypes.c_uint32), ("slots", ctypes.c_uint32), ("run", ctypes.c_uint32)]


class View(ctypes.Structure):
    _fields_ = [("mvp", ctypes.c_float * 16), ("w", ctypes.c_uint32), ("h", ctypes.c_uint32),
                ("variant", ctypes.c_int32), ("reserved", ctypes.c_uint32),
                ("fb", ctypes.c_void_p), ("rgba_out", ctypes.c_void_p)]


def _declare(lib):
    P, U32, U64, I32, SZ = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                            ctypes.c_size_t)
    sig = {
        "pcr_fb_bytes": (SZ, [U32, U32, I32]),
        "pcr_fb_clear": (I32, [P, U32, U32, I32, P]),
        "pcr_render": (I32, [P, U64, P, U32, U32, I32, P, P]),
        "pcr_render_ex": (I32, [P, U64, P, U32, U32, I32, P, P, P]),
        "pcr_resolve": (I32, [P, U32, U32, I32, P, P]),
        "pcr_resolve_raw": (I32, [P, U32, U32, I32, P, P]),
        "pcr_resolve_depth": (I32, [P, U32, U32, I32, I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    P, P, P]),
        "pcr_chunks_scratch_bytes": (SZ, [U32]),
        "pcr_render_chunks": (I32, [P, U32, P, U32, U32, I32, P, P, SZ, P, P]),
        "pcr_render_chunks_static": (I32, [P, U32, P, U32, U32, I32, P, P, P]),
        "pcr_reorder_scratch_bytes": (SZ, [U64, I32, U32]),
        "pcr_reorder": (I32, [P, P, P, U64, I32, U32, U64, P, SZ, P]),
        "pcr_batch_create": (I32, [P, P, U64, U32, P, P]),
        "pcr_batch_launch": (I32, [P, P, U32, P]),
        "pcr_batch_destroy": (I32, [P]),
        "pcr_render_batch": (I32, [P, U64, P, U32, P, P]),
        "pcr_release_batch_plans": (I32, []),
        "pcr_check_reciprocal": (I32, [U32, U32, P, P]),
        "pcr_count_visible": (I32, [P, U64, P, U32, U32, P, P]),
        "pcr_probe_atomics": (I32, [P, U64, I32, I32, U32, U32, U32, P, P]),
        "pcr_probe_read": (I32, [P, U64, U32, U32, P, P]),
        "pcr_last_error": (ctypes.c_char_p, []),
        "pcr_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def lib():
    """The loaded library (raises if it is not built).

    torch is imported first: its HIP runtime is then the one the dynamic
    loader binds libpcr's libamdhip64.so.7 to (same soname), so the library
    and torch share one runtime, its devices, streams and allocations.
    Loading libpcr first would put the whole process, torch included, on the
    system's runtime instead of the one torch was built with."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2104_07526_amd.build")
            import torch  # noqa: F401  (see above)
            _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _check(rc):
    if rc != OK:
        raise PcrError(rc, lib().pcr_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
    return getattr(stream, "cuda_stream", stream)


def _ptr(t):
    if t is None:
        return None
    return t.data_ptr() if hasattr(t, "data_ptr") else int(t)


def _fits(t, nbytes, what):
    """Raises ValueError when tensor ``t`` is not contiguous or holds fewer than
    ``nbytes`` bytes, before any device work is enqueued (the library takes
    raw addresses and cannot check; a raw address is the caller's
    responsibility)."""
    if t is None or not hasattr(t, "numel"):
        return
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{what} holds {have} bytes, {nbytes} needed")


def _fb_fits(fb, w, h, variant):
    # the size depends on the family and the robust HQ layout only
    need = int(lib().pcr_fb_bytes(w, h, variant & (0xFF | F_HQ_ROBUST))) if w > 0 and h > 0 else 0
    if need:                                # 0: invalid sizes, reported by the library call
        _fits(fb, need, "framebuffer")


def _npoints(points):
    if hasattr(points, "is_contiguous") and not points.is_contiguous():
        raise ValueError("points must be contiguous")
    nb = points.numel() * points.element_size()
    if nb % 16:
        raise ValueError("points must be 16-byte records")
    return nb // 16


def _mvp(m):
    a = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(16))
    return (ctypes.c_float * 16)(*a.tolist())


def _tune(t):
    if t is None:
        return None
    if isinstance(t, Tune):
        return ctypes.byref(t)
    return ctypes.byref(Tune(int(t.get("ppt", 0)), int(t.get("wg", 0)), int(t.get("grid", 0)),
                             int(t.get("group", 0)), int(t.get("slots", 0)), int(t.get("run", 0))))


# ---------------------------------------------------------------------------

def version() -> str:
    return lib().pcr_version().decode()


def check_reciprocal(first_bits, last_bits, stream=None):
    """(mismatches, bit sum mod 2^64, bit xor) of the projection reciprocal
    over the floats in the bit range (pcr_check_reciprocal; synchronises)."""
    import torch
    out = torch.zeros(3, dtype=torch.int64, device="cuda")
    _check(lib().pcr_check_reciprocal(first_bits, last_bits, _ptr(out), _stream(stream)))
    r = out.cpu().numpy().view(np.uint64)
    return int(r[0]), int(r[1]), int(r[2])


PROBE_RANDOM, PROBE_LINE, PROBE_ADDRESS, PROBE_CONTIGUOUS = 0, 1, 2, 3


def count_visible(points, mvp, w, h, stream=None) -> int:
    """Number of points the projection keeps for this view (synchronises)."""
    import torch
    out = torch.zeros(1, dtype=torch.int64, device=points.device)
    _check(lib().pcr_count_visible(_ptr(points), _npoints(points), _mvp(mvp), w, h, _ptr(out), _stream(stream)))
    return int(out.item())


def probe_atomics(buf, pattern, returning=False, workgroups=8192, iters=64, seed=1, sink=None, stream=None):
    """Enqueues the atomic-minimum throughput probe on the int64 tensor
    ``buf`` (its whole length rounded down to a multiple of 64 words).
    Returns the number of atomics it issues."""
    words = (buf.numel() * buf.element_size() // 8) // 64 * 64
    _check(lib().pcr_probe_atomics(_ptr(buf), words, pattern, int(bool(returning)), workgroups, iters, seed,
                                   _ptr(sink), _stream(stream)))
    return workgroups * 256 * iters


def probe_read(buf, per_thread=4, workgroups=4096, sink=None, stream=None):
    """Enqueues the read-rate probe over the tensor ``buf`` (its bytes taken
    as 16-byte records; a partial last record is left out).  ``sink``: an
    int32 device tensor (allocated if None).  Returns the bytes it reads."""
    import torch
    n16 = buf.numel() * buf.element_size() // 16
    if sink is None:
        sink = torch.zeros(1, dtype=torch.int32, device=buf.device)
    _fits(sink, 4, "sink")
    _check(lib().pcr_probe_read(_ptr(buf), n16, per_thread, workgroups, _ptr(sink), _stream(stream)))
    return 16 * n16


def fb_bytes(w, h, variant) -> int:
    return int(lib().pcr_fb_bytes(w, h, variant))


def alloc_fb(w, h, variant, device="cuda"):
    import torch
    nb = fb_bytes(w, h, variant)
    if nb == 0:
        raise PcrError(EINVAL, lib().pcr_last_error().decode())
    return torch.empty((nb + 7) // 8, dtype=torch.int64, device=device)


def fb_clear(fb, w, h, variant, stream=None):
    _fb_fits(fb, w, h, variant)
    _check(lib().pcr_fb_clear(_ptr(fb), w, h, variant, _stream(stream)))


def render(points, mvp, w, h, variant, fb, tune=None, stream=None, n=None):
    """Renders the 16-byte records of ``points`` (or the first ``n``)."""
    have = _npoints(points)
    n = have if n is None else n
    if n > have:
        raise ValueError(f"n = {n} but the buffer holds {have} points")
    _fb_fits(fb, w, h, variant)
    _check(lib().pcr_render_ex(_ptr(points), n, _mvp(mvp), w, h, variant, _ptr(fb), _tune(tune),
                               _stream(stream)))


def resolve(fb, w, h, variant, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty(w * h, dtype=torch.int32, device=fb.device)
    _fb_fits(fb, w, h, variant)
    _fits(out, 4 * w * h, "image")
    _check(lib().pcr_resolve(_ptr(fb), w, h, variant, _ptr(out), _stream(stream)))
    return out


def resolve_raw(fb, w, h, variant, out=None, stream=None):
    """The framebuffer's words in one linear layout (int64 tensor): the keys
    [w*h], or for HQ three planes [3*w*h] of depth bits, R<<32|G, B<<32|count."""
    import torch
    planes = 3 if (variant & 0xFF) == HQ else 1
    if out is None:
        out = torch.empty(planes * w * h, dtype=torch.int64, device=fb.device)
    _fb_fits(fb, w, h, variant)
    _fits(out, 8 * planes * w * h, "raw output")
    _check(lib().pcr_resolve_raw(_ptr(fb), w, h, variant, _ptr(out), _stream(stream)))
    return out


def chunks_scratch_bytes(nchunks) -> int:
    return int(lib().pcr_chunks_scratch_bytes(nchunks))


def chunk_table(chunks, device="cuda"):
    """Device array of pcr_chunk records from (buffer or device address, point
    count) pairs; a buffer may be a torch tensor (its data pointer is used)."""
    import torch
    rows = [[_ptr(b) or 0, int(n)] for b, n in chunks]
    return torch.tensor(rows if rows else [[0, 0]], dtype=torch.int64).to(device)


def render_chunks(table, nchunks, mvp, w, h, variant, fb, scratch=None, tune=None, stream=None):
    """Renders the first ``nchunks`` records of a device chunk table into fb
    (one launch per geometry pass).  Returns the scratch buffer."""
    import torch
    if scratch is None:
        scratch = torch.empty(max(chunks_scratch_bytes(nchunks), 256), dtype=torch.uint8, device=fb.device)
    nbytes = scratch.numel() * scratch.element_size()
    _fb_fits(fb, w, h, variant)
    _check(lib().pcr_render_chunks(_ptr(table), nchunks, _mvp(mvp), w, h, variant, _ptr(fb), _ptr(scratch),
                                   nbytes, _tune(tune), _stream(stream)))
    return scratch


STATIC_CHUNKS_MAX = 1 << 20


def render_chunks_static(table, nchunks, mvp, w, h, variant, fb, tune=None, stream=None):
    """render_chunks without a scratch buffer (pcr_render_chunks_static: the
    library's own per-GPU array; allocates nothing, calls on one GPU must not
    overlap)."""
    _fb_fits(fb, w, h, variant)
    _check(lib().pcr_render_chunks_static(_ptr(table), nchunks, _mvp(mvp), w, h, variant, _ptr(fb), _tune(tune),
                                          _stream(stream)))


def depth_coeffs(near, far, reverse=False):
    """(a, b) for DEPTH_HYPERBOLIC: window depth in [0,1] of a perspective
    projection with the given near and far planes (0 at near), or reverse-z
    (1 at near).  Computed in float64, rounded once to float32."""
    n, f = float(near), float(far)
    if reverse:
        a, b = -n / (f - n), f * n / (f - n)
    else:
        a, b = f / (f - n), -f * n / (f - n)
    return float(np.float32(a)), float(np.float32(b))


def resolve_depth(fb, w, h, variant, mode=DEPTH_LINEAR, a=0.0, b=0.0, empty=float("inf"), depth=None,
                  rgba=None, stream=None):
    """Depth image (float32 tensor [w*h]) and, when ``rgba`` is a tensor, the
    colour image in the same pass.  Returns (depth, rgba)."""
    import torch
    if depth is None:
        depth = torch.empty(w * h, dtype=torch.float32, device=fb.device)
    _fb_fits(fb, w, h, variant)
    _fits(depth, 4 * w * h, "depth image")
    _fits(rgba, 4 * w * h, "image")
    _check(lib().pcr_resolve_depth(_ptr(fb), w, h, variant, mode, a, b, empty, _ptr(rgba), _ptr(depth),
                                   _stream(stream)))
    return depth, rgba


def reorder_scratch_bytes(n, order, batch=128) -> int:
    return int(lib().pcr_reorder_scratch_bytes(n, order, batch))


def reorder(points, order, batch=128, seed=0, out=None, perm=None, want_perm=True, scratch=None,
            stream=None):
    """Returns (reordered points, permutation or None)."""
    import torch
    n = _npoints(points)
    if out is None:
        out = torch.empty_like(points)
    if want_perm and perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=points.device)
    need = reorder_scratch_bytes(n, order, batch)
    if scratch is None:
        scratch = torch.empty(max(need, 1), dtype=torch.uint8, device=points.device)
    nbytes = scratch.numel() * scratch.element_size()
    _fits(out, 16 * n, "output points")
    if want_perm:
        _fits(perm, 4 * n, "permutation")
    _check(lib().pcr_reorder(_ptr(points), _ptr(out), _ptr(perm) if want_perm else None, n, order,
                             batch, seed, _ptr(scratch), nbytes, _stream(stream)))
    return out, (perm if want_perm else None)


def make_view(mvp, w, h, variant, fb, rgba_out) -> View:
    """A batch view record.  It keeps references to ``fb`` and ``rgba_out``
    (the record itself only holds their device addresses), so the tensors
    live at least as long as the record; a launch that uses the record keeps
    them until the launch has completed on the device."""
    _fb_fits(fb, w, h, variant)
    _fits(rgba_out, 4 * w * h, "image")
    v = View()
    v.mvp[:] = [float(x) for x in np.asarray(mvp, np.float32).reshape(16)]
    v.w, v.h, v.variant = w, h, variant
    v.fb = _ptr(fb)
    v.rgba_out = _ptr(rgba_out)
    v._keep = (fb, rgba_out)
    return v


class _InFlight:
    """Buffers of enqueued launches, each held until the event recorded after
    its launch has completed (the library only sees raw device addresses, so
    a buffer dropped by the caller could otherwise be freed and reused while
    a kernel still writes it)."""

    def __init__(self):
        self._lock = threading.Lock()
        self._held = []

    def hold(self, event, refs):
        with self._lock:
            self._held = [(e, r) for e, r in self._held if not e.query()]
            self._held.append((event, refs))

    def pending(self):
        with self._lock:
            self._held = [(e, r) for e, r in self._held if not e.query()]
            return len(self._held)


def _held_refs(points, views):
    return (points, tuple(getattr(v, "_keep", ()) for v in views))


def _record(stream):
    import torch
    e = torch.cuda.Event()
    if stream is None:
        e.record()
    elif isinstance(stream, torch.cuda.Stream):
        e.record(stream)
    else:
        e.record(torch.cuda.ExternalStream(int(stream)))
    return e


_batch_inflight = _InFlight()


def render_batch(points, views, tune=None, stream=None):
    """One-call batch of pcr.View records over the library's plan cache
    (pcr_render_batch in include/pcr.h).  The views' buffers (and the points)
    are kept alive until the launch has completed."""
    arr = (View * max(1, len(views)))(*views)
    _check(lib().pcr_render_batch(_ptr(points), _npoints(points), arr, len(views), _tune(tune), _stream(stream)))
    _batch_inflight.hold(_record(stream), _held_refs(points, views))


def release_batch_plans():
    _check(lib().pcr_release_batch_plans())


class BatchPlan:
    """Renders up to ``capacity`` views of one resident cloud per launch, as a
    single hipGraph replay (pcr_batch_* in include/pcr.h)."""

    def __init__(self, points, capacity, tune=None, stream=None):
        self._points = points          # the plan keeps the device pointer
        self._inflight = _InFlight()
        self.capacity = capacity
        h = ctypes.c_void_p()
        _check(lib().pcr_batch_create(ctypes.byref(h), _ptr(points), _npoints(points), capacity,
                                      _tune(tune), _stream(stream)))
        self._h = h

    def launch(self, views, stream=None):
        """Enqueues one batch; the views' framebuffers and images are kept
        alive until it has completed on the device."""
        arr = (View * max(1, len(views)))(*views)
        _check(lib().pcr_batch_launch(self._h, arr, len(views), _stream(stream)))
        self._inflight.hold(_record(stream), _held_refs(None, views))

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().pcr_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
