#!/usr/bin/env python3
"""Benchmark of the compute point rasterizer on one MI355X.

Default workload (one "step"): a 100M-point LiDAR-like terrain (1 km x 1 km
heightfield, 16-byte points), 1920x1080 oblique view from 200 m, rendered by
the basic atomicMin renderer and by the deduplicating renderer, each on the
three vertex orders (scanline, Morton, Morton + shuffle in batches of 128):
six frames of clear + render + resolve.  Points are resident in HBM before
timing starts; the reorders are a one-time preprocessing step, timed apart.

Prints one JSON line.  `value` = points rendered per second over the timed
steps (billions/s).  `roofline` is for the kernel with the largest share of the
step time, timed with HIP events on the stream it runs on.  `cpu_baseline` is
the single-threaded CPU oracle on a bounded sample of the same work.

Other legs (one JSON line each, not part of the default run):
  --leg hq       300M-point building scene, high-quality blend, 2560x1440
  --leg big      796M-point cloud, 1920x1080, basic and dedup (shuffled Morton)
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

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE on
# the default workload (summaries under profiles/), scaled by the counters'
# reading for a plain 1 GiB copy (FETCH x2.0, WRITE x1.0).  Valid only for the
# kernel sources they were taken on: `src` is the sha256 of the render sources.
MEASURED_TRAFFIC = {
    # profiles/render_terrain100M_1080p.md
    "k_basic": {"src": "50c2301a3297d419da32128e6e87c94af63c4de08003e43ee1eaf9b94a4cc996",
                "fetch_bytes": 1670621757, "write_bytes": 1069193888},
    "k_dedup<u64>": {"src": "50c2301a3297d419da32128e6e87c94af63c4de08003e43ee1eaf9b94a4cc996",
                     "fetch_bytes": 1600064914, "write_bytes": 108992512},
}


def render_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("pcr_internal.h", "pcr_render.hip"):
        with open(os.path.join(ROOT, "paper_2104_07526_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(kernel):
    t = MEASURED_TRAFFIC.get(kernel)
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


def cpu_baseline(pts, m, W, H, frames_per_step, target_s=12.0):
    """The oracle (single thread) on a bounded sample of the step: the step's
    frames over a prefix of the cloud (the whole cloud, repeated, when it is
    fast enough), about `target_s` seconds of work."""
    import oracle
    orc = oracle.default()
    probe = min(len(pts), 2_000_000)
    t = time.perf_counter()
    fb = orc.render_basic(pts[:probe], m, W, H)
    orc.resolve_basic(fb, W, H)
    per_pt = (time.perf_counter() - t) / probe
    budget_pts = target_s / max(per_pt, 1e-12)
    n = int(min(len(pts), max(probe, budget_pts / frames_per_step)))
    reps = max(1, int(budget_pts // (n * frames_per_step)))
    t = time.perf_counter()
    for _ in range(reps * frames_per_step):
        fb = orc.render_basic(pts[:n], m, W, H)
        orc.resolve_basic(fb, W, H)
    dt = time.perf_counter() - t
    return {"value": round(n * frames_per_step * reps / dt / 1e9, 4), "unit": "Gpts/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{reps} x {frames_per_step} frames (render + resolve) of the first {n} points of the "
                      f"scanline-order cloud, {dt:.1f} s on one host core"}


def leg_main(args):
    import torch
    from paper_2104_07526_amd import pcr, synth
    n, W, H = args.n, 1920, 1080
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    timer.pairs.clear()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = e0.elapsed_time(e1)
    ms_step = total_ms / args.steps
    pts_per_step = n * len(keys)
    value = pts_per_step / (ms_step * 1e-3) / 1e9
    detail = {}
    kern_total = {}
    for o, v in keys:
        ks = timer.ms((o, v))
        med = float(np.median(ks))
        detail[f"{o}/{v}"] = {"render_ms": round(med, 4), "Gpts_s": round(n / med / 1e6, 2),
                              "GB_s": round(16 * n / med / 1e6, 1)}
        kern_total[v] = kern_total.get(v, 0.0) + sum(ks)
    # Dominant kernel: the variant whose render kernel takes the most time.
    dom = max(kern_total, key=kern_total.get)
    kname = {"basic": "k_basic", "dedup": "k_dedup<u64>"}
    dom_kernel = kname[dom]
    launches = len(keys) // len(variants) * args.steps
    avg_ms = kern_total[dom] / launches
    achieved = 16.0 * n / (avg_ms * 1e-3) / 1e9
    other = "dedup" if dom == "basic" else "basic"
    o_ms = kern_total[other] / launches
    o_ach = 16.0 * n / (o_ms * 1e-3) / 1e9
    best = min(detail.values(), key=lambda d: d["render_ms"])
    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64", "data": "synthetic",
        "config": {"workload": "terrain 100M points (16 B/point), 1920x1080 oblique view; basic and dedup "
                               "variants x scanline / Morton / Morton+shuffle-128 orders; frame = clear + "
                               "render + resolve",
                   "points": n, "resolution": [W, H], "frames_per_step": len(keys)},
        "roofline": {"bound": "hbm", "kernel": dom_kernel, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_for(dom_kernel),
                     "per_launch": f"16 B x {n} points = {16 * n / 1e9:.2f} GB, avg {avg_ms:.4f} ms over "
                                   f"the three orders"},
        "detail": {"frames": detail, "reorder_ms_100M": reorder_ms,
                   "roofline_" + other: {"bound": "hbm", "kernel": kname[other], "achieved": round(o_ach, 1),
                                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                         "frac": round(o_ach / HBM_PEAK_GBS, 4),
                                         "traffic": traffic_for(kname[other]), "avg_ms": round(o_ms, 4)},
                   "note": "k_basic issues one global 64-bit atomic per visible point; on MI355X such "
                           "atomics are performed memory-side at about 24-27 G/s for the whole chip, which "
                           "bounds the basic variant far below the HBM roofline",
                   "best_frame": {"Gpts_s": best["Gpts_s"], "GB_s": best["GB_s"],
                                  "hbm_frac": round(best["GB_s"] / HBM_PEAK_GBS, 4)},
                   "wall_s_timed": round(wall, 3),
                   "paper_context": "RTX 3090: 50 G points/s at 802 GB/s on a 796M-point scan (other "
                                    "hardware, other data)"},
    }
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(pts, m, W, H, len(keys))
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
                      ("hq_packed_plain", pcr.HQ | pcr.F_HQ_PACKED | pcr.F_PLAIN), ("dedup", pcr.DEDUP),
                      ("basic", pcr.BASIC)):
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
    HQ alternating: one autotuned batch plan (single hipGraph replay) against
    64 single-view renders in sequence; outputs compared for identity."""
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
    log("batch leg: autotuning the plan")
    pviews = [pcr.make_view(m, W, H, var, fb, im) for (m, W, H, var), fb, im in zip(views, fbs, imgs)]
    best_tune, table = tune.tune_batch(d, pviews, reps=2)
    log(f"batch leg: timing the tuned plan {best_tune}")
    plan = pcr.BatchPlan(d, len(pviews), tune=best_tune)
    bms = time_frames(lambda: plan.launch(pviews), args.steps, args.warmup)
    torch.cuda.synchronize()
    sequential(True)
    torch.cuda.synchronize()
    plan.launch(pviews)
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(imgs, ref))
    plan.close()
    pv = n * len(views)
    return {"metric": METRIC, "value": round(pv / bms / 1e6, 2), "unit": "Gpts/s (point-views)", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(bms, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+u64", "data": "synthetic",
            "config": {"workload": "145M points (terrain 100M + buildings 45M), shuffled Morton; 64 views, "
                                   "1280x720/1920x1080/3840x2160 cycling, basic/HQ alternating; one batch "
                                   "= clear + render + resolve of all 64 views", "points": n, "views": 64},
            "detail": {"batched_ms": round(bms, 3), "sequential_best_ms": round(seq_best, 3),
                       "sequential_plain_ms": round(seq_plain, 3),
                       "speedup_vs_sequential_best": round(seq_best / bms, 3),
                       "speedup_vs_sequential_plain": round(seq_plain / bms, 3),
                       "identical_images": bool(same), "tune": best_tune, "tune_table": table[:8],
                       "reorder_ms": round(rms, 2)}}


# Server policy of the serve leg (picked by sweeps on this load): batches that
# stream at least SERVE_BIG_POINTS points run one at a time (150M-1000M
# swept), a batch holds at most that many points x views, and at most
# SERVE_SMALL_BESIDE_BIG smaller batches run beside a large one (0, 2, 4 and
# no limit swept).
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
    policy = {"max_batch_points": SERVE_BIG_POINTS, "big_points": SERVE_BIG_POINTS,
              "small_beside_big": SERVE_SMALL_BESIDE_BIG}
    svc, rates = serve_measure(args, clouds, {"batched": ({}, policy)})
    # framebuffer budget sweep at the one-at-a-time rate (same policy)
    _, sweep = serve_measure(args, clouds, {f"budget_{b >> 20}MB": ({"budget_bytes": b}, policy)
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
                       "server": {"streams": 8, **policy},
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
        "dedup(LDS)": pcr.BASIC | pcr.F_LDS,
        "dedup": pcr.DEDUP,
        "dedup&early-z": pcr.DEDUP | pcr.F_LDS | pcr.F_REDUCE | pcr.F_EARLYZ,
        "HQ(plain)": pcr.HQ | pcr.F_PLAIN,
        "HQ": pcr.HQ,
        "HQ(packed)": pcr.HQ | pcr.F_HQ_PACKED,
    }
    poses = {"closeup": synth.terrain_closeup(W, H), "oblique": synth.terrain_oblique(W, H),
             "overview": synth.terrain_overview(W, H), "away": synth.terrain_away(W, H)}
    fbs = {fam: pcr.alloc_fb(W, H, fam) for fam in (pcr.BASIC, pcr.HQ)}
    img = torch.empty(W * H, dtype=torch.int32, device="cuda")
    ref = torch.empty(W * H, dtype=torch.int32, device="cuda")
    table, same = {}, True
    for oname, order in (("original", None), ("morton", pcr.ORDER_MORTON), ("shuffled", pcr.ORDER_SHUFFLE),
                         ("shuffled_morton", pcr.ORDER_MORTON_SHUFFLE)):
        d = base if order is None else pcr.reorder(base, order, 128, 3, want_perm=False)[0]
        torch.cuda.synchronize()
        for pname, m in poses.items():
            row = {}
            for tname, var in techniques.items():
                fam = pcr.HQ if (var & 0xFF) == pcr.HQ else pcr.BASIC
                fb = fbs[fam]
                layout = fam | (var & pcr.F_HQ_PACKED)      # clear and resolve follow the sums layout

                def frame():
                    pcr.fb_clear(fb, W, H, layout)
                    pcr.render(d, m, W, H, var, fb)
                    pcr.resolve(fb, W, H, layout, out=img)
                row[tname] = round(time_frames(frame, args.steps, args.warmup), 4)
                if tname == "atomicMin":
                    ref.copy_(img)
                elif fam != pcr.HQ:
                    same &= bool(torch.equal(img, ref))
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
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--leg", default="main", choices=["main", "hq", "big", "batch", "serve", "calib", "lod",
                                                        "resolve", "techniques"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
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
    legs = {"main": leg_main, "calib": leg_calib, "hq": leg_hq, "big": leg_big, "batch": leg_batch,
            "serve": leg_serve, "lod": leg_lod, "resolve": leg_resolve, "techniques": leg_techniques}
    if args.leg not in legs:
        print(f"leg {args.leg} is not available", file=sys.stderr)
        sys.exit(1)
    rec = legs[args.leg](args)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
