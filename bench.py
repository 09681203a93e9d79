#!/usr/bin/env python3
"""Benchmark of the compute point rasterizer on one MI355X.

Default workload (one "step"): the 796M-point building cloud (12.7 GB of
16-byte points, shuffled-Morton order), 1920x1080 overview of the whole scene,
rendered by the basic atomicMin renderer (Sec. 3.1: one global 64-bit atomic
per visible point) and by the deduplicating renderer (Sec. 3.3-3.4): two frames
of clear + render + resolve.  Points are resident in HBM before timing starts;
the reorder is a one-time preprocessing step, timed apart.

Prints one JSON line.  `value` = points rendered per second over the timed
steps (billions/s).  `roofline` is for the kernel with the largest share of the
step time (the basic kernel), timed with HIP events on the stream it runs on;
`roofline_atomic` puts the same kernel against the chip's measured atomic rate
(one atomic per visible point, counted on the device).  The detail holds the
deduplicating kernel's roofline, an HQ frame of the same cloud, the 100M-point
terrain frames and the atomic probe.  `cpu_baseline` is the single-threaded CPU
oracle on the same cloud and view.

Other legs (one JSON line each, not part of the default run):
  --leg terrain  100M terrain, 1920x1080: basic and dedup x three vertex orders
  --leg hq       300M-point building scene, high-quality blend, 2560x1440
  --leg big      796M-point cloud: dedup and HQ launch-shape autotuning
  --leg atomics  device-wide 64-bit atomicMin throughput by pattern and footprint
  --leg cpu      the CPU oracle on the full configured inputs
  --leg batch    64 views of a 145M-point cloud: batched plan vs single renders
  --leg serve    resident clouds + Poisson request load: p50/p99 latency
  --leg lod      level-of-detail frames: many chunks per frame in one launch
  --leg resolve  resolve with depth output (linear / window depth)
  --leg techniques  atomicMin / early-z / reduce / dedup / HQ x viewpoint x vertex order
  --leg calib    plain 1 GiB device copy (counter calibration for profiles)
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "billion points/s & HBM GB/s per frame; p50/p99 latency under request load"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch, keyed by (kernel, points), measured with rocprofv3
# --pmc FETCH_SIZE / WRITE_SIZE on the default workload (summaries under
# profiles/), scaled by the counters' reading for a plain 1 GiB copy (FETCH
# x2.0, WRITE x1.0).  Valid only for the kernel sources they were taken on:
# `src` is the sha256 of the render sources.
MEASURED_TRAFFIC = {
    # profiles/basic_dedup_796M_buildings_1080p.md (one dispatch each)
    ("k_basic", 796_000_000): {"src": "ff82f82c3c3becc0581d5b8b3b483e7ec2fd0022ca57b9fefe3e526737b655bd",
                                "fetch_bytes": 8423712 * 2048, "write_bytes": 23437392 * 1024},
    ("k_dedup<u64>", 796_000_000): {"src": "ff82f82c3c3becc0581d5b8b3b483e7ec2fd0022ca57b9fefe3e526737b655bd",
                                     "fetch_bytes": 6218804 * 2048, "write_bytes": 355971 * 1024},
    # profiles/render_terrain100M_1080p.md (averaged over the three orders)
    ("k_basic", 100_000_000): {"src": "ff82f82c3c3becc0581d5b8b3b483e7ec2fd0022ca57b9fefe3e526737b655bd",
                                "fetch_bytes": 889979 * 2048, "write_bytes": 1034719 * 1024},
    ("k_dedup<u64>", 100_000_000): {"src": "ff82f82c3c3becc0581d5b8b3b483e7ec2fd0022ca57b9fefe3e526737b655bd",
                                     "fetch_bytes": 781303 * 2048, "write_bytes": 106438 * 1024},
}


def render_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("pcr_internal.h", "pcr_render.hip"):
        with open(os.path.join(ROOT, "paper_2104_07526_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(kernel, n):
    t = MEASURED_TRAFFIC.get((kernel, n))
    if not t or t["src"] != render_sources_sha():
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ensure_built():
    from paper_2104_07526_amd import pcr
    if not os.path.exists(pcr.LIB_PATH):
        from paper_2104_07526_amd import build
        build.build()


def to_device(pts):
    import torch
    t = torch.from_numpy(pts.view(np.int32).reshape(-1, 4))
    return t.to("cuda", non_blocking=False)


class Timer:
    """HIP events on the current torch stream (the stream the library's
    kernels are enqueued on)."""

    def __init__(self):
        import torch
        self.torch = torch
        self.pairs = {}

    def start(self, key):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs.setdefault(key, []).append([e, None])

    def stop(self, key):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs[key][-1][1] = e

    def ms(self, key):
        return [a.elapsed_time(b) for a, b in self.pairs[key]]


def frame(pcr, d, m, W, H, variant, fb, out, timer, key):
    pcr.fb_clear(fb, W, H, variant)
    timer.start(key)
    pcr.render(d, m, W, H, variant, fb)
    timer.stop(key)
    pcr.resolve(fb, W, H, variant, out=out)


def host_info():
    """The host's CPU model (from /proc/cpuinfo, as lscpu shows it) and the
    number of CPUs this process may use (nproc)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"cpu_model": model, "nproc": nproc}


def cpu_baseline(pts, m, W, H, frames_per_step, what, target_s=12.0):
    """The oracle (single thread) on the step's closest-point frames: render +
    resolve over the whole cloud, repeated until about `target_s` seconds of
    work (at least the step's frames), or over a prefix of the cloud (for a
    shuffled order a spatially uniform sample) when one frame of the whole
    cloud would take longer.  Every closest-point variant has the same
    oracle."""
    import oracle
    orc = oracle.default()
    probe = min(len(pts), 2_000_000)
    t = time.perf_counter()
    fb = orc.render_basic(pts[:probe], m, W, H)
    orc.resolve_basic(fb, W, H)
    per_pt = (time.perf_counter() - t) / probe
    n = int(min(len(pts), max(probe, target_s / max(per_pt, 1e-12))))
    reps = 0
    t = time.perf_counter()
    while reps < frames_per_step or time.perf_counter() - t < target_s:
        fb = orc.render_basic(pts[:n], m, W, H)
        orc.resolve_basic(fb, W, H)
        reps += 1
    dt = time.perf_counter() - t
    scope = "the whole cloud" if n == len(pts) else f"the first {n} points"
    return {"value": round(n * reps / dt / 1e9, 4), "unit": "Gpts/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} frames (render + resolve) of {scope} of {what}, {dt:.1f} s on one host core; "
                      f"the step's {frames_per_step} closest-point frames are this same oracle computation",
            "host": host_info()}


def read_probe_rate(buf, reps=5):
    """Rate of the read probe over the resident tensor ``buf`` (GB/s, median
    of `reps` timed launches, the faster of two launch shapes), and its
    average launch time in ms."""
    import torch
    from paper_2104_07526_amd import pcr
    sink = torch.zeros(1, dtype=torch.int32, device=buf.device)
    best = None
    for per_thread, wgs in ((4, 4096), (8, 2048)):
        pcr.probe_read(buf, per_thread, wgs, sink)   # warm-up
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            nbytes = pcr.probe_read(buf, per_thread, wgs, sink)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        r = {"GB_s": round(nbytes / (float(np.median(ms)) * 1e-3) / 1e9, 1), "ms": round(float(np.median(ms)), 4),
             "per_thread": per_thread, "workgroups": wgs, "bytes": nbytes}
        if best is None or r["GB_s"] > best["GB_s"]:
            best = r
    return best


def probe_rate(pattern, words, returning=False, reps=3):
    """Device-wide atomicMin rate of one probe pattern (G atomics/s, median of
    `reps` launches timed with HIP events on the current stream)."""
    import torch
    from paper_2104_07526_amd import pcr
    buf = torch.full((words,), -1, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    pcr.probe_atomics(buf, pattern, returning, workgroups=2048, iters=8, sink=sink)   # warm-up
    rates = []
    for r in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ops = pcr.probe_atomics(buf, pattern, returning, seed=r + 2, sink=sink)
        e1.record()
        torch.cuda.synchronize()
        rates.append(ops / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del buf
    return float(np.median(rates))


PROBE_PATTERNS = {"random": 0, "line": 1, "address": 2, "contiguous": 3}


def terrain_frames(args, n, steps, warmup):
    """The 100M-point terrain frames: basic and dedup on the scanline, Morton
    and shuffled-Morton orders, 1920x1080 oblique view (times per frame)."""
    import torch
    from paper_2104_07526_amd import pcr, synth
    W, H = 1920, 1080
    t0 = time.perf_counter()
    pts = synth.terrain(n, seed=2)
    log(f"generated {n} terrain points in {time.perf_counter() - t0:.1f} s")
    m = synth.terrain_oblique(W, H)
    clouds = {"scanline": to_device(pts)}
    reorder_ms = {}
    for name, order in (("morton", pcr.ORDER_MORTON), ("morton_shuffle128", pcr.ORDER_MORTON_SHUFFLE)):
        scratch = torch.empty(pcr.reorder_scratch_bytes(n, order, 128), dtype=torch.uint8, device="cuda")
        out = torch.empty_like(clouds["scanline"])
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pcr.reorder(clouds["scanline"], order, 128, 3, out=out, want_perm=False, scratch=scratch)
            e1.record()
            torch.cuda.synchronize()
        reorder_ms[name] = round(e0.elapsed_time(e1), 3)
        clouds[name] = out
        del scratch
    variants = {"basic": pcr.BASIC, "dedup": pcr.DEDUP}
    fbs = {v: pcr.alloc_fb(W, H, var) for v, var in variants.items()}
    img = torch.empty(W * H, dtype=torch.int32, device="cuda")
    timer = Timer()
    keys = [(o, v) for o in clouds for v in variants]

    def step():
        for o, v in keys:
            frame(pcr, clouds[o], m, W, H, variants[v], fbs[v], img, timer, (o, v))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    timer.pairs.clear()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = e0.elapsed_time(e1) / steps
    detail, kern = {}, {}
    for o, v in keys:
        ks = timer.ms((o, v))
        med = float(np.median(ks))
        detail[f"{o}/{v}"] = {"render_ms": round(med, 4), "Gpts_s": round(n / med / 1e6, 2),
                              "GB_s": round(16 * n / med / 1e6, 1)}
        kern.setdefault(v, []).extend(ks)
    visible = {o: pcr.count_visible(clouds[o], m, W, H) for o in ("scanline",)}
    return {"pts": pts, "m": m, "keys": keys, "ms_step": ms_step, "wall": wall, "frames": detail,
            "kernel_ms": {v: float(np.mean(k)) for v, k in kern.items()}, "reorder_ms": reorder_ms,
            "visible": visible["scanline"]}


def leg_terrain(args):
    """The 100M-point terrain at 1920x1080 (oblique view): basic and dedup
    frames on the scanline, Morton and shuffled-Morton orders."""
    n, W, H = args.n, 1920, 1080
    r = terrain_frames(args, n, args.steps, args.warmup)
    value = n * len(r["keys"]) / (r["ms_step"] * 1e-3) / 1e9
    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["ms_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64", "data": "synthetic",
        "config": {"workload": "terrain 100M points (16 B/point), 1920x1080 oblique view; basic and dedup "
                               "variants x scanline / Morton / Morton+shuffle-128 orders; frame = clear + "
                               "render + resolve",
                   "points": n, "resolution": [W, H], "frames_per_step": len(r["keys"])},
        "detail": {"frames": r["frames"], "reorder_ms_100M": r["reorder_ms"],
                   "kernel_ms": {k: round(v, 4) for k, v in r["kernel_ms"].items()},
                   "visible_points_scanline": r["visible"], "wall_s_timed": round(r["wall"], 3)},
    }
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(r["pts"], r["m"], W, H, len(r["keys"]),
                                           "the 100M-point terrain (scanline order), oblique view")
    return rec


def leg_main(args):
    """The 796M-point building cloud (shuffled Morton), 1920x1080 overview:
    basic and dedup frames per step; HQ frame, terrain frames and the atomic
    probe in the detail."""
    import torch
    from paper_2104_07526_amd import pcr, synth
    n, W, H = args.big_n, 1920, 1080
    t0 = time.perf_counter()
    pts = synth.buildings(n, seed=4)
    log(f"generated {n} building points in {time.perf_counter() - t0:.1f} s")
    m = synth.buildings_overview(W, H, seed=4)
    d, rms = upload_reordered(pts, pcr.ORDER_MORTON_SHUFFLE)
    del pts
    log(f"uploaded and reordered (shuffled Morton) in {rms:.1f} ms of device time")
    variants = {"basic": pcr.BASIC, "dedup": pcr.DEDUP}
    fbs = {v: pcr.alloc_fb(W, H, var) for v, var in variants.items()}
    img = torch.empty(W * H, dtype=torch.int32, device="cuda")
    timer = Timer()

    def step():
        for v, var in variants.items():
            frame(pcr, d, m, W, H, var, fbs[v], img, timer, v)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    timer.pairs.clear()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = n * len(variants) / (ms_step * 1e-3) / 1e9
    kms = {v: float(np.mean(timer.ms(v))) for v in variants}
    frames = {v: {"render_ms": round(kms[v], 4), "Gpts_s": round(n / kms[v] / 1e6, 2),
                  "GB_s": round(16 * n / kms[v] / 1e6, 1), "hbm_frac": round(16 * n / kms[v] / 1e6 / HBM_PEAK_GBS, 4)}
              for v in variants}
    log(f"796M frames: {frames}")
    # Atomics of the basic frame: one per visible point.  Against the chip's
    # atomicMin rate, measured here by the probe at the framebuffer's footprint.
    visible = pcr.count_visible(d, m, W, H)
    words = W * H // 64 * 64
    probe = {name: round(probe_rate(p, words), 2) for name, p in PROBE_PATTERNS.items()}
    atom_rate = visible / (kms["basic"] * 1e-3) / 1e9
    # The practical floor of the point stream: the same buffer read once with
    # nothing else done (the deduplicating kernel's access pattern).
    read = read_probe_rate(d)
    # HQ frame of the same cloud (two passes over the points)
    fbh = pcr.alloc_fb(W, H, pcr.HQ)
    hq_timer = Timer()

    def hq_frame():
        frame(pcr, d, m, W, H, pcr.HQ, fbh, img, hq_timer, "hq")
    hq_ms = time_frames(hq_frame, max(3, args.steps // 2), 1)
    hq_kms = float(np.mean(hq_timer.ms("hq")[1:]))
    del fbh
    hq = {"frame_ms": round(hq_ms, 4), "render_ms": round(hq_kms, 4), "Gpts_s": round(n / hq_kms / 1e6, 2),
          "GB_s": round(32 * n / hq_kms / 1e6, 1), "hbm_frac": round(32 * n / hq_kms / 1e6 / HBM_PEAK_GBS, 4)}
    cpu = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        host_pts = d.cpu().numpy().reshape(-1).view(synth.POINT_DTYPE)
        log(f"downloaded the reordered cloud in {time.perf_counter() - t0:.1f} s")
        cpu = cpu_baseline(host_pts, m, W, H, len(variants),
                           f"the {n // 1_000_000}M-point building cloud in shuffled-Morton order, 1920x1080 overview")
        del host_pts
    del d, fbs
    torch.cuda.empty_cache()
    terrain = None
    if not args.no_terrain:
        r = terrain_frames(args, args.n, max(2, args.steps // 2), 1)
        terrain = {"workload": f"terrain {args.n // 1_000_000}M points, 1920x1080 oblique view, three orders",
                   "frames": r["frames"], "reorder_ms": r["reorder_ms"], "visible_points_scanline": r["visible"]}
        del r
    dom = max(kms, key=kms.get)
    kname = {"basic": "k_basic", "dedup": "k_dedup<u64>"}
    achieved = 16.0 * n / (kms[dom] * 1e-3) / 1e9
    other = "dedup" if dom == "basic" else "basic"
    o_ach = 16.0 * n / (kms[other] * 1e-3) / 1e9
    peak_atom = max(probe["random"], probe["address"])
    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64", "data": "synthetic",
        "config": {"workload": f"buildings {n // 1_000_000}M points (16 B/point, {16 * n / 1e9:.1f} GB), "
                               "shuffled Morton (batches of 128), 1920x1080 overview of the whole scene; basic "
                               "atomicMin and dedup frames; frame = clear + render + resolve",
                   "points": n, "resolution": [W, H], "frames_per_step": len(variants)},
        "roofline": {"bound": "hbm", "kernel": kname[dom], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_for(kname[dom], n),
                     "per_launch": f"16 B x {n} points = {16 * n / 1e9:.2f} GB, avg {kms[dom]:.4f} ms"},
        "roofline_atomic": {"bound": "atomic", "kernel": "k_basic", "achieved": round(atom_rate, 2),
                            "peak": round(peak_atom, 2), "unit": "G atomics/s",
                            "frac": round(atom_rate / peak_atom, 4),
                            "per_launch": f"{visible} visible points = {visible} global 64-bit atomicMin, avg "
                                          f"{kms['basic']:.4f} ms; peak = the probe's best rate with one atomic "
                                          f"per address (random or one address per wavefront) over the "
                                          f"{8 * words / 1e6:.1f} MB framebuffer"},
        "detail": {"frames": frames, "visible_points": visible,
                   "roofline_" + other: {"bound": "hbm", "kernel": kname[other], "achieved": round(o_ach, 1),
                                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                         "frac": round(o_ach / HBM_PEAK_GBS, 4),
                                         "traffic": traffic_for(kname[other], n), "avg_ms": round(kms[other], 4),
                                         "frac_of_read_probe": round(o_ach / read["GB_s"], 4)},
                   "read_probe": {**read, "note": "the cloud's buffer read once by pcr_probe_read (non-temporal "
                                                  "16-byte loads, no other work): the practical floor of a frame"},
                   "hq_frame": hq,
                   "atomic_probe_G_per_s": {**probe, "footprint_MB": round(8 * words / 1e6, 2)},
                   "reorder_ms": round(rms, 2),
                   "terrain_100M": terrain,
                   "note": "The 60% bar (the basic rasterizer at >= 60% of HBM bandwidth on the 796M cloud) "
                           "is not met: k_basic issues one device-scope 64-bit atomic per visible point, which "
                           "the chip performs memory-side at the probe's rate, far below the 300 G points/s "
                           "that 60% of HBM would need. The deduplicating kernel (detail) is the form that "
                           "approaches the HBM roofline.",
                   "wall_s_timed": round(wall, 3),
                   "paper_context": "RTX 3090: 50 G points/s at 802 GB/s on a 796M-point scan; atomicMin "
                                    "17.84 ms, dedup 15.26-18.01 ms (other hardware, other data)"},
    }
    if cpu is not None:
        rec["cpu_baseline"] = cpu
    return rec


def upload_reordered(pts, order=None, seed=3):
    """Host cloud -> device, optionally reordered on the GPU (one-time step)."""
    import torch
    from paper_2104_07526_amd import pcr
    d = to_device(pts)
    if order is None:
        return d, 0.0
    n = len(pts)
    scratch = torch.empty(pcr.reorder_scratch_bytes(n, order, 128), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(d)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    pcr.reorder(d, order, 128, seed, out=out, want_perm=False, scratch=scratch)
    e1.record()
    torch.cuda.synchronize()
    del scratch, d
    return out, e0.elapsed_time(e1)


def time_frames(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def leg_hq(args):
    """300M-point building scene, shuffled Morton, high-quality blend at
    2560x1440 (depth pass + colour pass + resolve), against the closest-point
    variants on the same frame."""
    import torch
    from paper_2104_07526_amd import pcr, synth
    n, W, H = 300_000_000, 2560, 1440
    t0 = time.perf_counter()
    pts = synth.buildings(n, seed=4)
    log(f"generated {n} building points in {time.perf_counter() - t0:.1f} s")
    m = synth.buildings_overview(W, H, seed=4)
    d, rms = upload_reordered(pts, pcr.ORDER_MORTON_SHUFFLE)
    del pts
    img = torch.empty(W * H, dtype=torch.int32, device="cuda")
    out, images = {}, {}
    for name, var in (("hq", pcr.HQ), ("hq_plain", pcr.HQ | pcr.F_PLAIN), ("hq_packed", pcr.HQ | pcr.F_HQ_PACKED),
                      ("hq_packed_plain", pcr.HQ | pcr.F_HQ_PACKED | pcr.F_PLAIN),
                      ("hq_robust", pcr.HQ | pcr.F_HQ_ROBUST), ("hq_robust_plain", pcr.HQ | pcr.F_HQ_ROBUST | pcr.F_PLAIN),
                      ("dedup", pcr.DEDUP), ("basic", pcr.BASIC)):
        fb = pcr.alloc_fb(W, H, var)

        def frame():
            pcr.fb_clear(fb, W, H, var)
            pcr.render(d, m, W, H, var, fb)
            pcr.resolve(fb, W, H, var, out=img)
        ms = time_frames(frame, args.steps, args.warmup)
        bpp = 32 if (var & 0xFF) == pcr.HQ else 16
        out[name] = {"frame_ms": round(ms, 4), "Gpts_s": round(n / ms / 1e6, 2),
                     "GB_s": round(bpp * n / ms / 1e6, 1), "hbm_frac": round(bpp * n / ms / 1e6 / HBM_PEAK_GBS, 4)}
        if name.startswith("hq"):
            images[name] = img.clone()
        del fb
    # pixels where the packed form differs from the two-word sums (more than
    # 1023 points blended into them)
    out["hq_packed"]["pixels_differing_from_hq"] = int((images["hq_packed"] != images["hq"]).sum())
    out["hq_packed"]["plain_same_image"] = bool(torch.equal(images["hq_packed"], images["hq_packed_plain"]))
    # the robust form equals the two-word form on every pixel
    out["hq_robust"]["same_image_as_hq"] = bool(torch.equal(images["hq_robust"], images["hq"]))
    out["hq_robust_plain"]["same_image_as_hq"] = bool(torch.equal(images["hq_robust_plain"], images["hq"]))
    return {"metric": METRIC, "value": out["hq"]["Gpts_s"], "unit": "Gpts/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": out["hq"]["frame_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64",
            "data": "synthetic",
            "config": {"workload": "buildings 300M points, shuffled Morton (batches of 128), 2560x1440, "
                                   "high-quality blend (epsilon 1%), frame = clear + 2 passes + resolve",
                       "points": n, "resolution": [W, H]},
            "detail": {"variants": out, "reorder_ms": round(rms, 2)}}


def leg_big(args):
    """The 796M-point cloud (12.7 GB), shuffled Morton, 1920x1080: basic,
    dedup and HQ frames."""
    import torch
    from paper_2104_07526_amd import pcr, synth
    n, W, H = 796_000_000, 1920, 1080
    t0 = time.perf_counter()
    pts = synth.buildings(n, seed=4)
    log(f"generated {n} building points in {time.perf_counter() - t0:.1f} s")
    m = synth.buildings_overview(W, H, seed=4)
    d, rms = upload_reordered(pts, pcr.ORDER_MORTON_SHUFFLE)
    del pts
    img = torch.empty(W * H, dtype=torch.int32, device="cuda")
    out = {}
    from paper_2104_07526_amd import tune
    runs = [("dedup", pcr.DEDUP, None), ("basic", pcr.BASIC, None), ("hq", pcr.HQ, None)]
    for name, var in (("dedup", pcr.DEDUP), ("hq", pcr.HQ)):
        fb = pcr.alloc_fb(W, H, var)
        best, _ = tune.tune_render(d, m, W, H, var, fb, reps=2, use_cache=False)
        runs.append((name + "_tuned", var, best))
        del fb
    for name, var, shape in runs:
        fb = pcr.alloc_fb(W, H, var)
        timer = Timer()

        def frame():
            pcr.fb_clear(fb, W, H, var)
            timer.start(name)
            pcr.render(d, m, W, H, var, fb, tune=shape)
            timer.stop(name)
            pcr.resolve(fb, W, H, var, out=img)
        ms = time_frames(frame, args.steps, args.warmup)
        kms = float(np.median(timer.ms(name)[args.warmup:]))
        bpp = 32 if (var & 0xFF) == pcr.HQ else 16
        out[name] = {"frame_ms": round(ms, 4), "render_ms": round(kms, 4), "Gpts_s": round(n / ms / 1e6, 2),
                     "GB_s": round(bpp * n / ms / 1e6, 1),
                     "render_hbm_frac": round(bpp * n / kms / 1e6 / HBM_PEAK_GBS, 4)}
        if shape:
            out[name]["shape"] = shape
        del fb
    return {"metric": METRIC, "value": out["dedup"]["Gpts_s"], "unit": "Gpts/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": out["dedup"]["frame_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64",
            "data": "synthetic",
            "config": {"workload": "buildings 796M points (12.7 GB), shuffled Morton, 1920x1080 overview; "
                                   "dedup (value, default launch shape), basic and HQ frames; dedup and HQ also "
                                   "with the autotuned shape", "points": n, "resolution": [W, H]},
            "detail": {"variants": out, "reorder_ms": round(rms, 2),
                       "paper_context": "RTX 3090, 796M-point scan: 15.26 ms (dedup, Morton), 17.84 ms "
                                        "(atomicMin, shuffled Morton)"}}


RES_CYCLE = [(1280, 720), (1920, 1080), (3840, 2160)]


def batch_views(count, seed=5):
    from paper_2104_07526_amd import pcr, synth
    views = []
    for i, (eye, tgt, up) in enumerate(synth.random_poses(count, seed=seed)):
        W, H = RES_CYCLE[i % 3]
        views.append((synth.mvp(eye, tgt, up, W, H), W, H, pcr.BASIC if i % 2 == 0 else pcr.HQ))
    return views


def leg_batch(args):
    """64 camera views of one 145M-point cloud (100M terrain + 45M buildings,
    shuffled Morton), framebuffers 1280x720 / 1920x1080 / 3840x2160, basic and
    HQ alternating: one batch plan (a single hipGraph replay) in its default
    shape (grouped passes: each tile of points loaded once per group of views)
    against 64 single-view renders in sequence with the same kernels, and the
    plan's per-view form; outputs compared for identity.  --tune also runs the
    autotuner over the plan shapes (not part of the default run)."""
    import torch
    from paper_2104_07526_amd import pcr, synth, tune
    nt, nb = 100_000_000, 45_000_000
    n = nt + nb
    t0 = time.perf_counter()
    pts = synth.terrain_and_buildings(nt, nb, seed=5)
    log(f"generated {n} points in {time.perf_counter() - t0:.1f} s")
    d, rms = upload_reordered(pts, pcr.ORDER_MORTON_SHUFFLE)
    del pts
    views = batch_views(64)
    fbs = [pcr.alloc_fb(W, H, var) for _, W, H, var in views]
    imgs = [torch.empty(W * H, dtype=torch.int32, device="cuda") for _, W, H, _ in views]
    ref = [torch.empty_like(i) for i in imgs]

    def sequential(best):
        for (m, W, H, var), fb, im in zip(views, fbs, ref):
            v = pcr.DEDUP if (best and var == pcr.BASIC) else var
            pcr.fb_clear(fb, W, H, v)
            pcr.render(d, m, W, H, v, fb)
            pcr.resolve(fb, W, H, v, out=im)
    log("batch leg: sequential single-view renders")
    seq_best = time_frames(lambda: sequential(True), max(1, args.steps // 2), 1)
    seq_plain = time_frames(lambda: sequential(False), 1, 0)
    sequential(True)
    torch.cuda.synchronize()
    pviews = [pcr.make_view(m, W, H, var, fb, im) for (m, W, H, var), fb, im in zip(views, fbs, imgs)]
    out = {}
    for name, shape in (("default", None), ("per_view", {"group": 1})):
        plan = pcr.BatchPlan(d, len(pviews), tune=shape)
        ms = time_frames(lambda: plan.launch(pviews), args.steps, args.warmup)
        for im in imgs:
            im.fill_(0)
        plan.launch(pviews)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(imgs, ref))
        plan.close()
        out[name] = {"ms": round(ms, 3), "identical_images": bool(same), "speedup_vs_sequential": round(seq_best / ms, 3)}
        log(f"batch leg: {name} plan {out[name]}")
    table = None
    if args.tune:
        log("batch leg: autotuning the plan")
        best_tune, table = tune.tune_batch(d, pviews, reps=2, use_cache=False)
        plan = pcr.BatchPlan(d, len(pviews), tune=best_tune)
        ms = time_frames(lambda: plan.launch(pviews), args.steps, args.warmup)
        plan.close()
        out["tuned"] = {"ms": round(ms, 3), "tune": best_tune, "speedup_vs_sequential": round(seq_best / ms, 3)}
    bms = out["default"]["ms"]
    pv = n * len(views)
    return {"metric": METRIC, "value": round(pv / bms / 1e6, 2), "unit": "Gpts/s (point-views)", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(bms, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64", "data": "synthetic",
            "config": {"workload": "145M points (terrain 100M + buildings 45M), shuffled Morton; 64 views, "
                                   "1280x720/1920x1080/3840x2160 cycling, basic/HQ alternating; one batch "
                                   "= clear + render + resolve of all 64 views", "points": n, "views": 64},
            "detail": {"plans": out, "sequential_ms": round(seq_best, 3),
                       "speedup_vs_sequential": out["default"]["speedup_vs_sequential"],
                       "sequential_note": "64 single-view renders, one after another, with the same kernels as "
                                          "the plan (dedup for basic views, the merged HQ passes)",
                       "sequential_atomicmin_ms": round(seq_plain, 3),
                       "tune_table": table[:8] if table else None, "reorder_ms": round(rms, 2)}}


# The earlier server policy, kept as the "overlap" comparison of the serve
# leg: batches that stream at least SERVE_BIG_POINTS points run one at a time,
# a batch holds at most that many points x views, and at most
# SERVE_SMALL_BESIDE_BIG smaller batches run beside a large one.
SERVE_BIG_POINTS = 250_000_000
SERVE_SMALL_BESIDE_BIG = 2

SERVE_SIZES = [10_000_000, 50_000_000, 100_000_000, 145_000_000, 300_000_000, 400_000_000, 500_000_000,
               796_000_000]


def serve_clouds(args):
    """The eight resident clouds (terrain and buildings alternating,
    shuffled-Morton order), scaled down by --n below 100M."""
    from paper_2104_07526_amd import pcr, synth
    sizes = SERVE_SIZES
    if args.n < 100_000_000:                         # reduced sizes for a quick run
        sizes = [max(1_000_000, s * args.n // 100_000_000) for s in sizes]
    clouds = []
    t0 = time.perf_counter()
    for i, sz in enumerate(sizes):
        gen = synth.terrain if i % 2 == 0 else synth.buildings
        pts = gen(sz, seed=10 + i)
        d, _ = upload_reordered(pts, pcr.ORDER_MORTON_SHUFFLE, seed=6)
        del pts
        clouds.append(d)
        log(f"cloud {i}: {sz} points resident ({time.perf_counter() - t0:.0f} s)")
    return sizes, clouds


def serve_measure(args, clouds, servers, fracs=(0.5, 0.8, 1.0, 1.25), seed=6):
    """Poisson request load at fractions of the one-at-a-time service rate.
    Every rate runs the one-at-a-time server and then each entry of
    `servers` ({name: (GpuBackend kwargs, Server kwargs)}) on the same arrival
    sequence; a sample of every server's images is checked against the
    one-at-a-time render."""
    import torch
    from paper_2104_07526_amd import pcr, synth
    from paper_2104_07526_amd.serve import GpuBackend, Request, Server, percentile
    res = [(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]
    rng = np.random.default_rng(seed)

    def make_requests(k):
        reqs = []
        poses = synth.random_poses(k, seed=int(rng.integers(1 << 30)))
        for (eye, tgt, up) in poses:
            c = int(rng.integers(0, len(clouds)))
            W, H = res[int(rng.integers(0, 4))]
            var = pcr.HQ if rng.random() < 0.3 else pcr.BASIC
            reqs.append(Request(c, synth.mvp(eye, tgt, up, W, H), W, H, var))
        return reqs
    budget = 2 << 30
    # One-at-a-time service: clear + render + resolve of one request, waited
    # for; basic requests use the deduplicating single-view path.
    fb = torch.empty(budget, dtype=torch.uint8, device="cuda")
    img = torch.empty(3840 * 2160, dtype=torch.int32, device="cuda")

    def plain(r, out=None):
        v = pcr.DEDUP if r.variant == pcr.BASIC else r.variant
        pcr.fb_clear(fb, r.w, r.h, v)
        pcr.render(clouds[r.cloud], r.mvp, r.w, r.h, v, fb)
        pcr.resolve(fb, r.w, r.h, v, out=img if out is None else out)
        torch.cuda.synchronize()
    cal = make_requests(200)
    for r in cal[:20]:
        plain(r)
    t = time.perf_counter()
    for r in cal:
        plain(r)
    svc = (time.perf_counter() - t) / len(cal)
    mu = 1.0 / svc
    nreq = args.requests
    backends = {name: GpuBackend(clouds, **{"budget_bytes": budget, "capacity": 16, **bk})
                for name, (bk, _) in servers.items()}
    # Keep the garbage collector out of the timed loops (both servers): the
    # objects created so far are frozen, and collection is paused meanwhile.
    gc.collect()
    gc.freeze()
    gc.disable()
    rates = {}
    for frac in fracs:
        lam = frac * mu
        reqs = make_requests(nreq)
        gaps = rng.exponential(1.0 / lam, nreq)
        pts_total = sum(pcr._npoints(clouds[r.cloud]) for r in reqs)
        # one-at-a-time server on this arrival sequence
        start = time.perf_counter() + 0.05
        arr = start + np.cumsum(gaps)
        lat_p = []
        for r, a in zip(reqs, arr):
            while time.perf_counter() < a:
                pass
            plain(r)
            lat_p.append(time.perf_counter() - a)
        wall_p = time.perf_counter() - start
        row = {"lambda_req_s": round(lam, 1),
               "plain": {"p50_ms": round(1e3 * percentile(lat_p, 50), 3),
                         "p99_ms": round(1e3 * percentile(lat_p, 99), 3),
                         "Gpts_s": round(pts_total / wall_p / 1e9, 2)}}
        for name, (_, sk) in servers.items():
            # continuous-batching server on the same sequence, driven inline by
            # the arrival loop (no second Python thread competing for the GIL)
            srv = Server(backends[name], budget_bytes=backends[name].arena_mem.numel(), **sk)
            start = time.perf_counter() + 0.05
            arr = start + np.cumsum(gaps)
            futs = []
            i = 0
            busy = True
            while i < nreq or busy:
                now = time.perf_counter()
                while i < nreq and arr[i] <= now:
                    reqs[i].arrival = float(arr[i])
                    futs.append(srv.submit(reqs[i]))
                    i += 1
                busy = srv.step()
            out = [f.result(timeout=600) for f in futs]
            wall_b = max(o.finished for o in out) - start
            lat_b = [o.latency for o in out]
            # identity: a sample of results against the one-at-a-time render
            chk = torch.empty(3840 * 2160, dtype=torch.int32, device="cuda")
            same = True
            for r, o in list(zip(reqs, out))[:: max(1, nreq // 20)]:
                plain(r, out=chk)
                same &= bool(torch.equal(o.image, chk[: r.w * r.h]))
            row[name] = {"p50_ms": round(1e3 * percentile(lat_b, 50), 3),
                         "p99_ms": round(1e3 * percentile(lat_b, 99), 3),
                         "Gpts_s": round(pts_total / wall_b / 1e9, 2),
                         "mean_batch": round(float(np.mean([o.batch_size for o in out])), 2),
                         "failed": sum(o.status != "ok" for o in out), "identical_sample": same}
        rates[f"{frac:.2f}"] = row
        log(f"rate {frac}: {row}")
    gc.enable()
    gc.unfreeze()
    for be in backends.values():
        be.close()
    return svc, rates


def leg_serve(args):
    """Eight resident clouds (10M-796M points, 36.8 GB), Poisson request load
    at fractions of the one-at-a-time service rate; continuous-batching server
    against a one-at-a-time server on the same arrival sequence."""
    sizes, clouds = serve_clouds(args)
    # The server: GpuBackend's defaults (two streams, one plan per cloud, no
    # cap on a batch's points), so that the requests of a cloud gather behind
    # its running batch and share the next one's point stream.  "overlap" is
    # the earlier policy: eight streams, two plans per cloud, batches capped
    # at SERVE_BIG_POINTS points x views, large batches one at a time.
    overlap = ({"streams": 8, "plans_per_cloud": 2},
               {"max_batch_points": SERVE_BIG_POINTS, "big_points": SERVE_BIG_POINTS,
                "small_beside_big": SERVE_SMALL_BESIDE_BIG})
    servers = {"batched": ({}, {}), "overlap": overlap}
    if args.serve_variants:
        servers["shared_3x1"] = ({"streams": 3, "plans_per_cloud": 1}, {})
        servers["shared_4x2"] = ({"streams": 4, "plans_per_cloud": 2}, {})
    svc, rates = serve_measure(args, clouds, servers)
    # framebuffer budget sweep at the one-at-a-time rate (same policy)
    _, sweep = serve_measure(args, clouds, {f"budget_{b >> 20}MB": ({"budget_bytes": b}, {})
                                            for b in (512 << 20, 8 << 30)}, fracs=(1.0,), seed=7)
    top = rates["1.00"]
    return {"metric": METRIC, "value": top["batched"]["Gpts_s"], "unit": "Gpts/s", "n_gpus": 1,
            "steps": args.requests, "warmup": 20, "ms_per_step": round(1e3 * svc, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64", "data": "synthetic",
            "config": {"workload": "8 resident clouds " + "/".join(f"{s // 1_000_000}M" for s in sizes) +
                                   "; Poisson arrivals at 0.5/0.8/1.0/1.25 x one-at-a-time rate; requests: "
                                   "random cloud, pose, 720p-4K, basic/HQ 70/30; 2 GB framebuffer budget (0.5 GB and "
                                   "8 GB at the one-at-a-time rate in the detail)",
                       "requests_per_rate": args.requests},
            "detail": {"service_ms_one_at_a_time": round(1e3 * svc, 3), "rates": rates,
                       "budget_sweep_at_1.0": sweep["1.00"],
                       "server": {"streams": 2, "plans_per_cloud": 1, "plan": "grouped passes (default shape)"},
                       "p50_ms_at_1.0": top["batched"]["p50_ms"], "p99_ms_at_1.0": top["batched"]["p99_ms"]}}


def lod_chunks(n, mean, rng):
    """Chunk sizes of an LPC-style octree with about `mean` points per node:
    log-normal sizes (sigma 0.8, mean `mean`) cut to sum exactly to n."""
    sizes = []
    left = n
    mu = np.log(mean) - 0.8 ** 2 / 2
    while left > 0:
        s = int(min(left, max(1, rng.lognormal(mu, 0.8))))
        sizes.append(s)
        left -= s
    return np.array(sizes, np.int64)


def leg_lod(args):
    """Level-of-detail frames (Sec. 5.4): many separate point buffers per
    frame.  One chunked launch per pass against one pcr_render per chunk (eager
    and captured in a hipGraph) and against one render of the same points as a
    single buffer.  The paper's 4M-point cases (1624 chunks of ~2.4k, 80 of
    ~49.4k) on a 4M-point sphere scan stand-in, and 100M terrain points in
    chunks of ~2.4k.  Chunks are contiguous Morton ranges (octree nodes), drawn
    in shuffled table order; frame = clear + render + resolve, 1920x1080."""
    import ctypes

    import torch
    from paper_2104_07526_amd import pcr, synth
    W, H = 1920, 1080
    rng = np.random.default_rng(12)
    cases = [("sphere 4M, 1624 chunks ~2.4k", "sphere", 4_000_000, 2_463),
             ("sphere 4M, 80 chunks ~49.4k", "sphere", 4_000_000, 50_000),
             ("terrain 100M, chunks ~2.4k", "terrain", 100_000_000, 2_400)]
    L = pcr.lib()
    out = {}
    for name, kind, n, mean in cases:
        pts = synth.sphere(n, seed=1) if kind == "sphere" else synth.terrain(n, seed=2)
        m = synth.sphere_view(W, H) if kind == "sphere" else synth.terrain_oblique(W, H)
        d, _ = upload_reordered(pts, pcr.ORDER_MORTON)
        del pts
        sizes = lod_chunks(n, mean, rng)
        offs = np.concatenate([[0], np.cumsum(sizes)])
        order = rng.permutation(len(sizes))
        base = d.data_ptr()
        table = [(base + 16 * int(offs[c]), int(sizes[c])) for c in order]
        tab = pcr.chunk_table(table)
        scratch = torch.empty(max(256, pcr.chunks_scratch_bytes(len(table))), dtype=torch.uint8, device="cuda")
        var = pcr.DEDUP
        fb = pcr.alloc_fb(W, H, var)
        img = torch.empty(W * H, dtype=torch.int32, device="cuda")
        mvp_c = (ctypes.c_float * 16)(*[float(x) for x in np.asarray(m, np.float32).reshape(16)])
        fbp = fb.data_ptr()
        timer = Timer()

        def chunked():
            pcr.fb_clear(fb, W, H, var)
            timer.start("k")
            pcr.render_chunks(tab, len(table), m, W, H, var, fb, scratch=scratch)
            timer.stop("k")
            pcr.resolve(fb, W, H, var, out=img)

        def per_chunk():
            pcr.fb_clear(fb, W, H, var)
            s = torch.cuda.current_stream().cuda_stream
            for addr, cnt in table:
                L.pcr_render(addr, cnt, mvp_c, W, H, var, fbp, s)
            pcr.resolve(fb, W, H, var, out=img)

        def single():
            pcr.fb_clear(fb, W, H, var)
            pcr.render(d, m, W, H, var, fb)
            pcr.resolve(fb, W, H, var, out=img)

        res = {"chunks": len(table), "points": n, "mean_chunk": round(n / len(table), 1)}
        ms = time_frames(chunked, args.steps, args.warmup)
        kms = float(np.median(timer.ms("k")[args.warmup:]))
        ref = img.clone()
        res["chunked"] = {"frame_ms": round(ms, 4), "fps": round(1e3 / ms, 1), "render_ms": round(kms, 4),
                          "Gpts_s": round(n / kms / 1e6, 2), "GB_s": round(16 * n / kms / 1e6, 1),
                          "hbm_frac": round(16 * n / kms / 1e6 / HBM_PEAK_GBS, 4)}
        steps_pc = max(1, min(args.steps, 3)) if len(table) > 10_000 else args.steps
        ms = time_frames(per_chunk, steps_pc, 1)
        same = bool(torch.equal(img, ref))
        res["per_chunk_launches"] = {"frame_ms": round(ms, 4), "fps": round(1e3 / ms, 1), "identical": same}
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            per_chunk()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            per_chunk()
        ms = time_frames(g.replay, steps_pc, 1)
        same = bool(torch.equal(img, ref))
        res["per_chunk_graph"] = {"frame_ms": round(ms, 4), "fps": round(1e3 / ms, 1), "identical": same}
        del g
        ms = time_frames(single, args.steps, args.warmup)
        res["single_buffer"] = {"frame_ms": round(ms, 4), "fps": round(1e3 / ms, 1),
                                "identical": bool(torch.equal(img, ref))}
        # The same points as one buffer in the table's draw order: separates
        # the cost of the chunk table from that of the shuffled chunk order.
        # Gathered on the host (a device index_select of this size returned
        # a wrong gather on this stack; the leg checks the image below).
        idx = np.concatenate([np.arange(offs[c], offs[c] + sizes[c]) for c in order])
        dt = torch.from_numpy(d.cpu().numpy()[idx]).to(d.device)
        del idx

        def single_table_order():
            pcr.fb_clear(fb, W, H, var)
            pcr.render(dt, m, W, H, var, fb)
            pcr.resolve(fb, W, H, var, out=img)
        ms = time_frames(single_table_order, args.steps, args.warmup)
        res["single_buffer_table_order"] = {"frame_ms": round(ms, 4), "fps": round(1e3 / ms, 1),
                                            "identical": bool(torch.equal(img, ref))}
        del dt
        out[name] = res
        log(f"lod {name}: {res}")
        del d, tab, fb
        torch.cuda.empty_cache()
    top = out[cases[0][0]]
    return {"metric": METRIC, "value": top["chunked"]["fps"], "unit": "frames/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": top["chunked"]["frame_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64",
            "data": "synthetic",
            "config": {"workload": "level-of-detail frames: many separate point buffers (Morton-range chunks, "
                                   "shuffled draw order), dedup, 1920x1080; value = frames/s of the 4M-point, "
                                   "1624-chunk case", "resolution": [W, H]},
            "detail": {"cases": out,
                       "paper_context": "RTX 3090, 4M-point lion in 1624 nodes: 500 FPS compute (718 GL_POINTS); "
                                        "80 nodes: 2096 FPS compute"}}


def leg_techniques(args):
    """The update techniques of Sec. 3 against viewpoint and vertex order
    (the structure of the paper's detailed tables, Sec. 5.2-5.3): every
    technique renders the same 100M-point terrain frames (clear + render +
    resolve, 1920x1080) from a close-up, the oblique view, an overview and a
    pose with no point in the frustum (the streaming floor), in the original
    (scanline), Morton, shuffled and shuffled-Morton orders.  Every technique
    of one frame gives the same image (checked here on each frame)."""
    import torch
    from paper_2104_07526_amd import pcr, synth
    n, W, H = args.n, 1920, 1080
    pts = synth.terrain(n, seed=2)
    base = to_device(pts)
    del pts
    techniques = {
        "atomicMin": pcr.BASIC,
        "early-z": pcr.BASIC | pcr.F_EARLYZ,
        "reduce": pcr.BASIC | pcr.F_REDUCE,
        "reduce&early-z": pcr.BASIC | pcr.F_REDUCE | pcr.F_EARLYZ,
        "reduce(wave)": pcr.BASIC | pcr.F_REDUCE_WAVE,
        "reduce(pairs)": pcr.BASIC | pcr.F_REDUCE_PAIR,
        "dedup(LDS)": pcr.BASIC | pcr.F_LDS,
        "dedup": pcr.DEDUP,
        "dedup&early-z": pcr.DEDUP | pcr.F_LDS | pcr.F_REDUCE | pcr.F_EARLYZ,
        "HQ(plain)": pcr.HQ | pcr.F_PLAIN,
        "HQ": pcr.HQ,
        "HQ(packed)": pcr.HQ | pcr.F_HQ_PACKED,
        "HQ(robust)": pcr.HQ | pcr.F_HQ_ROBUST,
    }
    poses = {"closeup": synth.terrain_closeup(W, H), "oblique": synth.terrain_oblique(W, H),
             "overview": synth.terrain_overview(W, H), "away": synth.terrain_away(W, H)}
    fbs = {pcr.BASIC: pcr.alloc_fb(W, H, pcr.BASIC), pcr.HQ: pcr.alloc_fb(W, H, pcr.HQ | pcr.F_HQ_ROBUST)}
    img = torch.empty(W * H, dtype=torch.int32, device="cuda")
    ref = torch.empty(W * H, dtype=torch.int32, device="cuda")
    hq_ref = torch.empty(W * H, dtype=torch.int32, device="cuda")
    table, same, hq_same = {}, True, True
    for oname, order in (("original", None), ("morton", pcr.ORDER_MORTON), ("shuffled", pcr.ORDER_SHUFFLE),
                         ("shuffled_morton", pcr.ORDER_MORTON_SHUFFLE)):
        d = base if order is None else pcr.reorder(base, order, 128, 3, want_perm=False)[0]
        torch.cuda.synchronize()
        for pname, m in poses.items():
            row = {}
            for tname, var in techniques.items():
                fam = pcr.HQ if (var & 0xFF) == pcr.HQ else pcr.BASIC
                fb = fbs[fam]
                layout = fam | (var & (pcr.F_HQ_PACKED | pcr.F_HQ_ROBUST))   # clear and resolve follow the sums layout

                def frame():
                    pcr.fb_clear(fb, W, H, layout)
                    pcr.render(d, m, W, H, var, fb)
                    pcr.resolve(fb, W, H, layout, out=img)
                row[tname] = round(time_frames(frame, args.steps, args.warmup), 4)
                if tname == "atomicMin":
                    ref.copy_(img)
                elif fam != pcr.HQ:
                    same &= bool(torch.equal(img, ref))
                elif tname == "HQ(plain)":
                    hq_ref.copy_(img)
                elif tname != "HQ(packed)":          # the packed form differs past 1023 points per pixel
                    hq_same &= bool(torch.equal(img, hq_ref))
            table.setdefault(oname, {})[pname] = row
            log(f"{oname} {pname}: {row}")
        if order is not None:
            del d
    best = table["shuffled_morton"]["oblique"]["dedup"]
    return {"metric": METRIC, "value": round(n / best / 1e6, 2), "unit": "Gpts/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": best, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64", "data": "synthetic",
            "config": {"workload": f"terrain {n // 1_000_000}M points, 1920x1080; techniques x poses "
                                   "(close-up, oblique, overview, no point in frustum) x orders (original, "
                                   "Morton, shuffled, shuffled Morton); frame = clear + render + resolve; value: "
                                   "dedup, oblique view, shuffled Morton"},
            "detail": {"frame_ms": table, "closest_point_images_identical": same,
                       "hq_images_identical_plain_merged_robust": hq_same,
                       "paper_context": "RTX 3090, 145M-point town scan, shuffled Morton: atomicMin 3.75 ms, "
                                        "early-z 3.46, reduce 3.39, reduce&early-z 3.31, dedup 3.44, HQS 7.08"}}


def leg_resolve(args):
    """Resolve passes on rendered frames: colour only, and colour + depth
    (linear and window depth) in one pass, basic and HQ at 1080p and 4K."""
    import torch
    from paper_2104_07526_amd import pcr, synth
    pts = synth.terrain(20_000_000, seed=2)
    d = to_device(pts)
    del pts
    out = {}
    for W, H in ((1920, 1080), (3840, 2160)):
        m = synth.terrain_oblique(W, H)
        a, b = pcr.depth_coeffs(0.5, 5000.0)
        for var, vname in ((pcr.DEDUP, "basic"), (pcr.HQ, "hq")):
            fb = pcr.alloc_fb(W, H, var)
            pcr.fb_clear(fb, W, H, var)
            pcr.render(d, m, W, H, var, fb)
            img = torch.empty(W * H, dtype=torch.int32, device="cuda")
            dep = torch.empty(W * H, dtype=torch.float32, device="cuda")
            px = W * H
            # bytes per pixel read + written: basic key 8; HQ depth 4, sums 16; colour 4; depth 4
            hq = var == pcr.HQ
            runs = {"colour": (lambda: pcr.resolve(fb, W, H, var, out=img), 20 if hq else 12),
                    "colour+linear_depth": (lambda: pcr.resolve_depth(fb, W, H, var, pcr.DEPTH_LINEAR, depth=dep,
                                                                     rgba=img), 28 if hq else 16),
                    "colour+window_depth": (lambda: pcr.resolve_depth(fb, W, H, var, pcr.DEPTH_HYPERBOLIC, a, b,
                                                                     depth=dep, rgba=img), 28 if hq else 16),
                    "window_depth": (lambda: pcr.resolve_depth(fb, W, H, var, pcr.DEPTH_HYPERBOLIC, a, b,
                                                              depth=dep), 8 if hq else 12)}
            for rname, (fn, bpp) in runs.items():
                ms = time_frames(fn, max(20, args.steps * 5), args.warmup)
                out[f"{W}x{H}/{vname}/{rname}"] = {"ms": round(ms, 4), "bytes_per_pixel": bpp,
                                                    "GB_s": round(bpp * px / ms / 1e6, 1)}
            del fb
    return {"metric": METRIC, "value": out["1920x1080/basic/colour+window_depth"]["GB_s"], "unit": "GB/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": out["1920x1080/basic/colour+window_depth"]["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64+f32", "data": "synthetic",
            "config": {"workload": "resolve of a rendered 20M-point terrain frame, 1080p and 4K, basic and HQ: "
                                   "colour, colour + depth (linear / window), depth only"},
            "detail": out}


def leg_atomics(args):
    """Device-wide 64-bit atomicMin throughput (the operation of the basic
    renderer) by access pattern, framebuffer footprint (720p, 1080p, 1440p and
    4K u64 framebuffers, and 1 GB) and returning / fire-and-forget form."""
    foot = {"720p": 1280 * 720, "1080p": 1920 * 1080, "1440p": 2560 * 1440, "4K": 3840 * 2160,
            "1GB": (1 << 30) // 8}
    table = {}
    for fname, px in foot.items():
        words = px // 64 * 64
        for ret in (False, True):
            row = {name: round(probe_rate(p, words, ret), 2) for name, p in PROBE_PATTERNS.items()}
            table[f"{fname}/{'returning' if ret else 'no_return'}"] = {**row, "footprint_MB": round(8 * words / 1e6, 2)}
            log(f"atomics {fname} returning={ret}: {row}")
    top = table["1080p/no_return"]
    return {"metric": "device-wide 64-bit atomicMin rate", "value": top["random"], "unit": "G atomics/s",
            "n_gpus": 1, "steps": 3, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "2048-8192 workgroups x 256 lanes x 8-64 atomicMin each; patterns: random "
                                   "word per lane, 8 lanes per 64-byte line, one word per wavefront, 64 "
                                   "consecutive words per wavefront; value: random words over a 1080p u64 "
                                   "framebuffer (16.6 MB), no return"},
            "detail": table}


def leg_cpu(args):
    """The single-threaded CPU oracle on the full configured inputs: the 1M
    sphere (720p), the 100M terrain (scanline order, 1080p oblique), the 300M
    building scene (HQ, shuffled Morton, 1440p) and the 796M building cloud
    (basic, shuffled Morton, 1080p overview).  Reordered clouds are reordered on
    the GPU and downloaded before timing.  Times are render + resolve."""
    import oracle
    from paper_2104_07526_amd import pcr, synth
    orc = oracle.default()
    out = {}

    def timed(fn):
        t = time.perf_counter()
        fn()
        return time.perf_counter() - t

    def reordered(pts):
        d, _ = upload_reordered(pts, pcr.ORDER_MORTON_SHUFFLE)
        h = d.cpu().numpy().reshape(-1).view(synth.POINT_DTYPE)
        del d
        return h

    pts = synth.sphere(1_000_000, seed=1)
    m = synth.sphere_view(1280, 720)
    dt = timed(lambda: orc.resolve_basic(orc.render_basic(pts, m, 1280, 720), 1280, 720))
    out["sphere_1M_720p_basic"] = {"s": round(dt, 3), "Gpts_s": round(1e6 / dt / 1e9, 4)}
    log(f"cpu: {out}")
    pts = synth.terrain(100_000_000, seed=2)
    m = synth.terrain_oblique(1920, 1080)
    dt = timed(lambda: orc.resolve_basic(orc.render_basic(pts, m, 1920, 1080), 1920, 1080))
    out["terrain_100M_scanline_1080p_basic"] = {"s": round(dt, 3), "Gpts_s": round(1e8 / dt / 1e9, 4)}
    log(f"cpu: {out}")
    del pts
    pts = reordered(synth.buildings(300_000_000, seed=4))
    m = synth.buildings_overview(2560, 1440, seed=4)

    def hq():
        _, RG, BA = orc.render_hq(pts, m, 2560, 1440)
        orc.resolve_hq(RG, BA, 2560, 1440)
    dt = timed(hq)
    out["buildings_300M_shuffled_morton_1440p_hq"] = {"s": round(dt, 3), "Gpts_s": round(3e8 / dt / 1e9, 4)}
    log(f"cpu: {out}")
    del pts
    pts = reordered(synth.buildings(796_000_000, seed=4))
    m = synth.buildings_overview(1920, 1080, seed=4)
    dt = timed(lambda: orc.resolve_basic(orc.render_basic(pts, m, 1920, 1080), 1920, 1080))
    out["buildings_796M_shuffled_morton_1080p_basic"] = {"s": round(dt, 3), "Gpts_s": round(7.96e8 / dt / 1e9, 4)}
    log(f"cpu: {out}")
    del pts
    top = out["buildings_796M_shuffled_morton_1080p_basic"]
    return {"metric": METRIC, "value": top["Gpts_s"], "unit": "Gpts/s", "n_gpus": 0, "steps": 1, "warmup": 0,
            "ms_per_step": round(1e3 * top["s"], 1), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+u64", "data": "synthetic",
            "config": {"workload": "CPU oracle, one thread, full inputs: 1M sphere 720p basic; 100M terrain "
                                   "1080p basic; 300M buildings 1440p HQ; 796M buildings 1080p basic"},
            "detail": {"runs": out, "cores": 1, "host": host_info()}}


def leg_calib(args):
    """A plain device-to-device copy of 1 GiB: reference for FETCH_SIZE and
    WRITE_SIZE counters."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"metric": "copy GB/s (calibration)", "value": round(2 * nbytes / ms / 1e6, 1), "unit": "GB/s",
            "bytes_read": nbytes, "bytes_written": nbytes, "ms": round(ms, 4)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000_000, help="terrain points (terrain, techniques legs)")
    ap.add_argument("--big-n", type=int, default=796_000_000, help="points of the default leg's building cloud")
    ap.add_argument("--leg", default="main", choices=["main", "terrain", "hq", "big", "atomics", "cpu", "batch",
                                                        "serve", "calib", "lod", "resolve", "techniques"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-terrain", action="store_true", help="default leg: skip the terrain frames")
    ap.add_argument("--tune", action="store_true", help="batch leg: also run the plan autotuner")
    ap.add_argument("--serve-variants", action="store_true", help="serve leg: also measure other server policies")
    ap.add_argument("--requests", type=int, default=2000, help="requests per arrival rate (serve leg)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the renderer runs on a single MI355X here "
              "(multi-GPU sharding is described in the design notes, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ensure_built()
    legs = {"main": leg_main, "terrain": leg_terrain, "atomics": leg_atomics, "cpu": leg_cpu,
            "calib": leg_calib, "hq": leg_hq, "big": leg_big, "batch": leg_batch,
            "serve": leg_serve, "lod": leg_lod, "resolve": leg_resolve, "techniques": leg_techniques}
    if args.leg not in legs:
        print(f"leg {args.leg} is not available", file=sys.stderr)
        sys.exit(1)
    rec = legs[args.leg](args)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
