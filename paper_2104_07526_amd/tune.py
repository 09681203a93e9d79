"""Autotuner for the render launch shapes.

Times candidate shapes (points per thread, LDS slots, views per point pass)
on the caller's actual workload and returns the fastest; results are cached
in a JSON file keyed by device, workload kind, point-count class and view mix,
so a later process reuses them without re-timing.
"""
from __future__ import annotations

import json
import math
import os
import sys
import threading

from . import pcr

CACHE = os.environ.get("PCR_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "pcr_tune.json"))
_lock = threading.Lock()

# group 1: each view its own single-view pass inside the plan's graph, with
# points per thread 1-16 and workgroups of 64-1024 threads (tiles of at most
# 4096 points, whose LDS tables fit); group > 1: the grouped passes (each tile
# loaded once per group of views), views per group 2-32, one-wavefront
# workgroups with 2-8 points per thread.
BATCH_CANDIDATES = ([{"ppt": p, "group": 1, "wg": w} for p in (1, 2, 4, 8, 16) for w in (64, 256, 1024)
                     if p * w <= 4096] +
                    [{"ppt": p, "group": g, "wg": 64} for p in (2, 4, 8) for g in (2, 4, 8, 16, 32)])
RENDER_CANDIDATES = [{"ppt": p, "wg": w, "slots": s} for p in (4, 8, 16) for w in (64, 128, 256, 512)
                     for s in (0, 512, 1024, 2048)]


def _device():
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key, value):
    with _lock:
        data = _load()
        data[key] = value
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE + ".tmp", "w") as f:
                json.dump(data, f, indent=1)
            os.replace(CACHE + ".tmp", CACHE)
        except OSError:
            pass


def _key(kind, n, mix):
    return f"{_device()}|{kind}|n~2^{int(math.log2(max(n, 1)))}|{mix}"


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_batch(points, views, candidates=None, reps=2, use_cache=True):
    """(best tune dict, [(ms, tune), ...] sorted) for a batch of pcr.View."""
    n = pcr._npoints(points)
    mix = "v%d-hq%d-px%d" % (len(views), sum(v.variant == pcr.HQ for v in views),
                             int(math.log2(max(1, sum(v.w * v.h for v in views)))))
    key = _key("batch", n, mix)
    if use_cache:
        hit = _load().get(key)
        if hit:
            return hit["tune"], hit["table"]
    table = []
    for c in candidates or BATCH_CANDIDATES:
        print(f"tune_batch: {c}", file=sys.stderr, flush=True)
        try:
            plan = pcr.BatchPlan(points, len(views), tune=c)
        except pcr.PcrError:
            continue                     # shape does not fit (LDS)
        try:
            ms = _time(lambda: plan.launch(views), reps)
        finally:
            plan.close()
        table.append((round(ms, 4), dict(c)))
    table.sort(key=lambda t: t[0])
    best = table[0][1]
    _store(key, {"tune": best, "table": table})
    return best, table


def tune_render(points, mvp, w, h, variant, fb, candidates=None, reps=3, use_cache=True):
    """(best tune dict, table) for single-view renders of one variant."""
    n = pcr._npoints(points)
    key = _key("render", n, f"{variant}-{w}x{h}")
    if use_cache:
        hit = _load().get(key)
        if hit:
            return hit["tune"], hit["table"]
    table = []
    for c in candidates or RENDER_CANDIDATES:
        def frame():
            pcr.fb_clear(fb, w, h, variant)
            pcr.render(points, mvp, w, h, variant, fb, tune=c)
        try:
            ms = _time(frame, reps)
        except pcr.PcrError:
            continue                     # shape does not fit (LDS)
        table.append((round(ms, 4), dict(c)))
    table.sort(key=lambda t: t[0])
    best = table[0][1]
    _store(key, {"tune": best, "table": table})
    return best, table
