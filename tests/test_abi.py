"""The C ABI without a GPU: the library loads, exports every entry point that
include/pcr.h declares, and rejects bad arguments on the host before any HIP
call.  No compute call is made here."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2104_07526_amd import pcr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcr.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pcr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("pcr_fb_bytes", "pcr_fb_clear", "pcr_render", "pcr_render_ex", "pcr_resolve", "pcr_resolve_depth",
              "pcr_reorder_scratch_bytes", "pcr_reorder", "pcr_batch_create", "pcr_batch_launch",
              "pcr_batch_destroy", "pcr_last_error", "pcr_version", "pcr_resolve_raw"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = pcr.lib()
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", pcr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (pcr_\w+)", out))
    assert set(declared()) <= exported


def test_header_compiles_as_c():
    src = '#include "pcr.h"\nint main(void){ pcr_point p; (void)p; return (int)sizeof(pcr_point) - 16; }\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), "-x", "c", "-",
                        "-o", "/dev/null"], input=src, text=True, capture_output=True)
    assert r.returncode == 0, r.stderr


def test_fb_bytes():
    assert pcr.fb_bytes(1920, 1080, pcr.BASIC) == 8 * 1920 * 1080
    assert pcr.fb_bytes(1920, 1080, pcr.DEDUP | pcr.F_LDS) == 8 * 1920 * 1080
    d = (4 * 1920 * 1080 + 255) // 256 * 256
    assert pcr.fb_bytes(1920, 1080, pcr.HQ) == d + 16 * 1920 * 1080
    assert pcr.fb_bytes(3, 1, pcr.HQ) == 256 + 48
    for bad in [(0, 5, 0), (5, 0, 0), (1 << 24, 1, 0), (70000, 70000, 0), (4, 4, 7), (4, 4, pcr.BASIC | pcr.F_HQ_DEPTH)]:
        assert pcr.fb_bytes(*bad) == 0, bad


@pytest.mark.parametrize("variant,msg", [
    (3, "unknown variant"),
    (pcr.BASIC | (1 << 20), "flag bits"),
    (pcr.DEDUP | pcr.F_HQ_COLOR, "flag bits"),
    (pcr.DEDUP | pcr.F_PLAIN | pcr.F_LDS, "PLAIN"),
    (pcr.BASIC | pcr.F_PLAIN | pcr.F_REDUCE_WAVE, "PLAIN"),
    (pcr.HQ | pcr.F_PLAIN | pcr.F_REDUCE_PAIR, "PLAIN"),
    (pcr.BASIC | pcr.F_LDS | pcr.F_REDUCE_PAIR, "PAIR"),
    (pcr.HQ | pcr.F_LDS | pcr.F_REDUCE_PAIR, "PAIR"),
])
def test_render_rejects_bad_variants(variant, msg):
    m = (ctypes.c_float * 16)()
    rc = pcr.lib().pcr_render(None, 0, m, 4, 4, variant, None, None)
    assert rc == pcr.EINVAL
    assert msg in pcr.lib().pcr_last_error().decode()


def test_packed_hq_flag_checks():
    """PCR_F_HQ_PACKED belongs to PCR_HQ only; chunked frames of the other
    variants refuse it before touching any pointer."""
    L = pcr.lib()
    m = (ctypes.c_float * 16)()
    assert L.pcr_fb_bytes(64, 32, pcr.HQ | pcr.F_HQ_PACKED) == L.pcr_fb_bytes(64, 32, pcr.HQ)
    assert L.pcr_fb_bytes(64, 32, pcr.DEDUP | pcr.F_HQ_PACKED) == 0
    assert L.pcr_render(None, 0, m, 4, 4, pcr.BASIC | pcr.F_HQ_PACKED, None, None) == pcr.EINVAL
    assert "flag bits" in L.pcr_last_error().decode()
    assert L.pcr_render_chunks(16, 3, m, 4, 4, pcr.DEDUP | pcr.F_HQ_PACKED, 16, 256, 256, None, None) in (
        pcr.EUNSUPPORTED, pcr.EINVAL)


def test_render_rejects_bad_pointers_and_sizes():
    L = pcr.lib()
    m = (ctypes.c_float * 16)()
    assert L.pcr_render(None, 0, m, 0, 4, 0, 16, None) == pcr.EINVAL
    assert L.pcr_render(None, 10, m, 4, 4, 0, 16, None) == pcr.EINVAL          # null points
    assert L.pcr_render(8, 10, m, 4, 4, 0, 16, None) == pcr.EINVAL             # misaligned points
    assert L.pcr_render(16, 10, m, 4, 4, 0, 8, None) == pcr.EINVAL             # misaligned fb
    assert L.pcr_render(16, 10, None, 4, 4, 0, 16, None) == pcr.EINVAL         # null mvp
    tune = pcr.Tune(3, 256, 0, 0, 0)
    assert L.pcr_render_ex(16, 10, m, 4, 4, 0, 16, ctypes.byref(tune), None) == pcr.EINVAL
    tune = pcr.Tune(4, 96, 0, 0, 0)
    assert L.pcr_render_ex(16, 10, m, 4, 4, 0, 16, ctypes.byref(tune), None) == pcr.EINVAL
    assert L.pcr_resolve(16, 4, 4, 0, None, None) == pcr.EINVAL
    assert L.pcr_resolve_depth(16, 4, 4, 0, 0, 0.0, 0.0, 0.0, None, None, None) == pcr.EINVAL  # no depth_out
    assert L.pcr_resolve_depth(16, 4, 4, 0, 2, 0.0, 0.0, 0.0, None, 16, None) == pcr.EINVAL    # mode
    assert "mode" in L.pcr_last_error().decode()
    assert L.pcr_resolve_depth(16, 4, 4, 0, 1, 0.0, 0.0, 0.0, 18, 16, None) == pcr.EINVAL      # rgba align
    assert L.pcr_resolve_depth(16, 4, 4, 0, 1, 0.0, 0.0, 0.0, None, 18, None) == pcr.EINVAL    # depth align
    assert L.pcr_resolve_depth(8, 4, 4, 0, 1, 0.0, 0.0, 0.0, None, 16, None) == pcr.EINVAL     # fb align
    assert L.pcr_resolve_depth(16, 4, 4, 7, 1, 0.0, 0.0, 0.0, None, 16, None) == pcr.EINVAL    # variant
    assert L.pcr_fb_clear(None, 4, 4, 0, None) == pcr.EINVAL
    assert L.pcr_resolve_raw(16, 4, 4, 0, None, None) == pcr.EINVAL                     # no raw_out
    assert L.pcr_resolve_raw(16, 4, 4, pcr.HQ, 12, None) == pcr.EINVAL                  # raw_out align
    assert L.pcr_resolve_raw(8, 4, 4, 0, 16, None) == pcr.EINVAL                        # fb align
    assert L.pcr_resolve_raw(16, 0, 4, 0, 16, None) == pcr.EINVAL                       # size
    assert L.pcr_resolve_raw(16, 4, 4, pcr.HQ | pcr.F_HQ_PACKED | pcr.F_HQ_ROBUST, 16, None) == pcr.EINVAL


def test_chunk_argument_checks():
    L = pcr.lib()
    m = (ctypes.c_float * 16)()
    assert L.pcr_chunks_scratch_bytes(0) == 0
    assert L.pcr_chunks_scratch_bytes((1 << 24) + 1) == 0
    assert L.pcr_chunks_scratch_bytes(1) == 256 + 4 * (1 << 17)       # offsets, then one word per workgroup
    assert L.pcr_chunks_scratch_bytes(100) == 1024 + 4 * (1 << 17)
    # nothing to draw: accepted without touching any pointer
    assert L.pcr_render_chunks(None, 0, m, 4, 4, pcr.DEDUP, 16, None, 0, None, None) == pcr.OK
    assert L.pcr_render_chunks(None, 3, m, 4, 4, pcr.DEDUP, 16, 256, 256, None, None) == pcr.EINVAL
    assert L.pcr_render_chunks(16, 3, m, 4, 4, pcr.DEDUP, 16, None, 256, None, None) == pcr.EINVAL
    assert L.pcr_render_chunks(16, 3, m, 4, 4, pcr.DEDUP, 16, 256, 16, None, None) == pcr.ENOMEM
    assert L.pcr_render_chunks(16, 3, None, 4, 4, pcr.DEDUP, 16, 256, 256, None, None) == pcr.EINVAL
    assert L.pcr_render_chunks(16, 3, m, 4, 4, pcr.DEDUP, 8, 256, 256, None, None) == pcr.EINVAL
    assert L.pcr_render_chunks(16, (1 << 24) + 1, m, 4, 4, pcr.DEDUP, 16, 256, 1 << 30, None, None) == pcr.EINVAL
    for v in (pcr.BASIC | pcr.F_EARLYZ, pcr.DEDUP | pcr.F_LDS, pcr.HQ | pcr.F_PLAIN, pcr.DEDUP | pcr.F_HQ_DEPTH):
        assert L.pcr_render_chunks(16, 3, m, 4, 4, v, 16, 256, 256, None, None) in (pcr.EUNSUPPORTED, pcr.EINVAL)
    assert L.pcr_render_chunks(16, 3, m, 4, 4, pcr.BASIC | pcr.F_EARLYZ, 16, 256, 256, None, None) == \
        pcr.EUNSUPPORTED
    for v in (pcr.BASIC | pcr.F_REDUCE_WAVE, pcr.HQ | pcr.F_REDUCE_PAIR):
        assert L.pcr_render_chunks(16, 3, m, 4, 4, v, 16, 256, 256, None, None) == pcr.EUNSUPPORTED


def test_render_batch_argument_checks():
    L = pcr.lib()
    assert L.pcr_render_batch(16, 100, None, 0, None, None) == pcr.OK          # nothing to do
    assert L.pcr_render_batch(16, 100, None, 3, None, None) == pcr.EINVAL
    assert L.pcr_release_batch_plans() == pcr.OK


def test_reorder_argument_checks():
    L = pcr.lib()
    assert L.pcr_reorder_scratch_bytes(1000, 5, 128) == 0
    assert L.pcr_reorder_scratch_bytes(1000, pcr.ORDER_MORTON_SHUFFLE, 0) == 0
    assert L.pcr_reorder_scratch_bytes(1 << 32, pcr.ORDER_MORTON, 128) == 0
    a = L.pcr_reorder_scratch_bytes(1000, pcr.ORDER_MORTON, 128)
    b = L.pcr_reorder_scratch_bytes(1000, pcr.ORDER_MORTON_SHUFFLE, 128)
    assert 0 < a < b
    assert L.pcr_reorder(16, 16 * 2000, None, 1000, 9, 128, 0, 256, a, None) == pcr.EINVAL
    assert L.pcr_reorder(16, 16 * 2000, None, 1 << 32, 0, 128, 0, 256, a, None) == pcr.EINVAL
    assert L.pcr_reorder(16, 32, None, 1000, 0, 128, 0, 256, a, None) == pcr.EINVAL     # overlap
    assert L.pcr_reorder(16, 16 * 2000, None, 1000, 0, 128, 0, 256, a - 1, None) == pcr.ENOMEM
    assert L.pcr_reorder(16, 16 * 2000, None, 0, 0, 128, 0, 0, 0, None) == pcr.OK       # n == 0


def test_batch_argument_checks():
    L = pcr.lib()
    h = ctypes.c_void_p()
    assert L.pcr_batch_create(ctypes.byref(h), 16, 100, 0, None, None) == pcr.EINVAL
    assert L.pcr_batch_create(ctypes.byref(h), 8, 100, 4, None, None) == pcr.EINVAL
    assert L.pcr_batch_create(ctypes.byref(h), 16, 0, 4, None, None) == pcr.EINVAL
    tune = pcr.Tune(3, 64, 0, 4, 0)           # points per thread not a power of two
    assert L.pcr_batch_create(ctypes.byref(h), 16, 100, 4, ctypes.byref(tune), None) == pcr.EINVAL
    assert "points per thread" in L.pcr_last_error().decode()
    tune = pcr.Tune(8, 64, 0, 4, 0, 12)       # run not a multiple of ppt
    assert L.pcr_batch_create(ctypes.byref(h), 16, 100, 4, ctypes.byref(tune), None) == pcr.EINVAL
    assert "run" in L.pcr_last_error().decode()
    assert L.pcr_batch_launch(None, None, 0, None) == pcr.EINVAL
    assert L.pcr_batch_destroy(None) == pcr.OK


def test_binding_checks_tensor_sizes_before_enqueueing():
    """The binding refuses tensors too small (or not contiguous) for the
    buffers the library would write, before any call reaches the device."""
    import torch
    W, H = 64, 32
    m = np.eye(4, dtype=np.float32)
    pts = torch.zeros(100, 4, dtype=torch.int32)
    small_fb = torch.zeros(pcr.fb_bytes(W, H, pcr.BASIC) // 8 - 1, dtype=torch.int64)
    with pytest.raises(ValueError, match="framebuffer"):
        pcr.fb_clear(small_fb, W, H, pcr.BASIC)
    with pytest.raises(ValueError, match="framebuffer"):
        pcr.render(pts, m, W, H, pcr.DEDUP | pcr.F_EARLYZ, small_fb)
    hq_fb = torch.zeros(pcr.fb_bytes(W, H, pcr.BASIC) // 8, dtype=torch.int64)   # basic-sized, HQ needs more
    with pytest.raises(ValueError, match="framebuffer"):
        pcr.resolve(hq_fb, W, H, pcr.HQ, out=torch.zeros(W * H, dtype=torch.int32))
    fb = torch.zeros(pcr.fb_bytes(W, H, pcr.BASIC) // 8, dtype=torch.int64)
    with pytest.raises(ValueError, match="points"):
        pcr.render(pts, m, W, H, pcr.BASIC, fb, n=101)
    with pytest.raises(ValueError, match="image"):
        pcr.resolve(fb, W, H, pcr.BASIC, out=torch.zeros(W * H - 1, dtype=torch.int32))
    with pytest.raises(ValueError, match="contiguous"):
        pcr.resolve(fb, W, H, pcr.BASIC, out=torch.zeros(W * H, 2, dtype=torch.int32)[:, 0])
    with pytest.raises(ValueError, match="depth image"):
        pcr.resolve_depth(fb, W, H, pcr.BASIC, depth=torch.zeros(W * H - 1, dtype=torch.float32))
    with pytest.raises(ValueError, match="output points"):
        pcr.reorder(pts, pcr.ORDER_MORTON, out=torch.zeros(99, 4, dtype=torch.int32), want_perm=False,
                    scratch=torch.zeros(1 << 20, dtype=torch.uint8))
    with pytest.raises(ValueError, match="permutation"):
        pcr.reorder(pts, pcr.ORDER_MORTON, perm=torch.zeros(99, dtype=torch.int32),
                    scratch=torch.zeros(1 << 20, dtype=torch.uint8))
    with pytest.raises(ValueError, match="image"):
        pcr.make_view(m, W, H, pcr.BASIC, fb, torch.zeros(W * H - 1, dtype=torch.int32))
    strided = torch.zeros(4, 100, dtype=torch.int32).t()          # 100 records, column-major
    expanded = torch.zeros(1, 4, dtype=torch.int32).expand(100, 4)  # 100 records over 16 bytes
    for bad in (strided, expanded):
        with pytest.raises(ValueError, match="points must be contiguous"):
            pcr.render(bad, m, W, H, pcr.BASIC, fb)
        with pytest.raises(ValueError, match="points must be contiguous"):
            pcr.reorder(bad, pcr.ORDER_MORTON, want_perm=False, scratch=torch.zeros(1 << 20, dtype=torch.uint8))


def test_measurement_helpers_check_arguments():
    """pcr_count_visible, pcr_probe_atomics and pcr_probe_read refuse bad
    arguments on the host (no GPU call is made for them)."""
    L = pcr.lib()
    m = (ctypes.c_float * 16)()
    assert L.pcr_count_visible(None, 0, m, 0, 4, 8, None) == pcr.EINVAL
    assert L.pcr_count_visible(None, 0, m, 4, 4, None, None) == pcr.EINVAL
    assert L.pcr_count_visible(None, 0, None, 4, 4, 8, None) == pcr.EINVAL
    assert L.pcr_count_visible(8, 5, m, 4, 4, 8, None) == pcr.EINVAL      # misaligned points
    assert L.pcr_count_visible(None, 0, m, 4, 4, 8, None) == pcr.OK       # n == 0: nothing to do
    for words in (0, 63, 65, 1 << 32):
        assert L.pcr_probe_atomics(64, words, 0, 0, 1, 1, 0, None, None) == pcr.EINVAL
    assert L.pcr_probe_atomics(32, 64, 0, 0, 1, 1, 0, None, None) == pcr.EINVAL   # misaligned buffer
    assert L.pcr_probe_atomics(64, 64, 4, 0, 1, 1, 0, None, None) == pcr.EINVAL   # unknown pattern
    assert L.pcr_probe_atomics(64, 64, 0, 1, 1, 1, 0, None, None) == pcr.EINVAL   # returning without sink
    assert L.pcr_probe_atomics(64, 64, 0, 0, 0, 1, 0, None, None) == pcr.EINVAL   # no workgroups
    assert L.pcr_probe_read(None, 0, 4, 1, None, None) == pcr.OK                   # n16 == 0: nothing to do
    assert L.pcr_probe_read(None, 4, 4, 1, 64, None) == pcr.EINVAL                 # no buffer
    assert L.pcr_probe_read(72, 4, 4, 1, 64, None) == pcr.EINVAL                   # misaligned buffer
    for per_thread in (0, 1, 2, 16):
        assert L.pcr_probe_read(64, 4, per_thread, 1, 64, None) == pcr.EINVAL
    for wgs in (0, (1 << 22) + 1):
        assert L.pcr_probe_read(64, 4, 4, wgs, 64, None) == pcr.EINVAL
    assert L.pcr_probe_read(64, 4, 4, 1, None, None) == pcr.EINVAL                 # no sink
    assert L.pcr_probe_read(64, 4, 4, 1, 66, None) == pcr.EINVAL                   # misaligned sink


def test_static_chunks_refuse_too_many_chunks():
    """pcr_render_chunks_static refuses more chunks than its array holds, and
    its other checks match pcr_render_chunks (host only, nothing enqueued)."""
    L = pcr.lib()
    m = (ctypes.c_float * 16)()
    assert L.pcr_render_chunks_static(16, pcr.STATIC_CHUNKS_MAX + 1, m, 4, 4, pcr.DEDUP, 16, None, None) == pcr.EINVAL
    assert "chunks" in L.pcr_last_error().decode()
    assert L.pcr_render_chunks_static(16, 3, m, 4, 4, pcr.DEDUP | pcr.F_EARLYZ, 16, None, None) == pcr.EUNSUPPORTED
    assert L.pcr_render_chunks_static(16, 3, m, 4, 4, pcr.DEDUP, None, None, None) == pcr.EINVAL
    assert L.pcr_render_chunks_static(None, 3, m, 4, 4, pcr.DEDUP, 16, None, None) == pcr.EINVAL
    assert L.pcr_render_chunks_static(None, 0, m, 4, 4, pcr.DEDUP, 16, None, None) == pcr.OK


def test_robust_hq_flag_checks():
    """PCR_F_HQ_ROBUST belongs to PCR_HQ, excludes PCR_F_HQ_PACKED, and adds
    one 8-byte fast word per pixel to the framebuffer."""
    L = pcr.lib()
    m = (ctypes.c_float * 16)()
    RB = pcr.HQ | pcr.F_HQ_ROBUST
    assert L.pcr_fb_bytes(64, 32, RB) == L.pcr_fb_bytes(64, 32, pcr.HQ) + 8 * 64 * 32
    assert L.pcr_fb_bytes(64, 32, pcr.DEDUP | pcr.F_HQ_ROBUST) == 0
    assert L.pcr_fb_bytes(64, 32, RB | pcr.F_HQ_PACKED) == 0
    assert L.pcr_render(None, 0, m, 4, 4, RB | pcr.F_HQ_PACKED, None, None) == pcr.EINVAL
    assert "pick one" in L.pcr_last_error().decode()
    assert L.pcr_render(None, 0, m, 4, 4, pcr.BASIC | pcr.F_HQ_ROBUST, None, None) == pcr.EINVAL
