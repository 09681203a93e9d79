"""The serving workload at its full size: eight resident clouds of 10M, 50M,
100M, 145M, 300M, 400M, 500M and 796M points (terrain and buildings
alternating, shuffled Morton, 36.8 GB in HBM), Poisson request arrivals served
by the continuous-batching server while earlier batches are still on the GPU
(a burst, then Poisson arrivals; 720p to 4K, basic / HQ 70 / 30, 2 GB
framebuffer budget).  Every served image
equals the same request rendered alone, and one request per cloud (a 4K HQ view
of the 796M cloud among them) equals the CPU oracle."""
import time

import numpy as np
import pytest

from paper_2104_07526_amd import pcr, synth
from paper_2104_07526_amd.serve import GpuBackend, Request, Server

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(1200)]

SIZES = [10_000_000, 50_000_000, 100_000_000, 145_000_000, 300_000_000, 400_000_000, 500_000_000, 796_000_000]
RES = [(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]


def log(msg):
    print(f"[serve-fullsize] {msg}", flush=True)


def requests(k, nclouds, seed):
    rng = np.random.default_rng(seed)
    out = []
    for eye, tgt, up in synth.random_poses(k, seed=seed):
        c = int(rng.integers(0, nclouds))
        w, h = RES[int(rng.integers(0, len(RES)))]
        var = pcr.HQ if rng.random() < 0.3 else pcr.BASIC
        out.append(Request(c, synth.mvp(eye, tgt, up, w, h), w, h, var))
    return out


def test_served_results_at_full_size(orc):
    import torch
    host, dev = [], []
    t0 = time.perf_counter()
    for i, n in enumerate(SIZES):
        gen = synth.terrain if i % 2 == 0 else synth.buildings
        pts = gen(n, seed=10 + i)
        d = torch.from_numpy(pts.view(np.int32).reshape(-1, 4)).to("cuda")
        msh, _ = pcr.reorder(d, pcr.ORDER_MORTON_SHUFFLE, 128, 6, want_perm=False)
        torch.cuda.synchronize()
        del d
        host.append(pts)
        dev.append(msh)
        log(f"cloud {i}: {n} points resident ({time.perf_counter() - t0:.0f} s)")
    assert sum(16 * len(h) for h in host) == 16 * sum(SIZES)
    reqs = requests(240, len(SIZES), seed=61)
    # one request per cloud for the oracle; the last is a 4K HQ view of the 796M cloud
    pick = {}
    for k, r in enumerate(reqs):
        pick.setdefault(r.cloud, k)
    assert len(pick) == len(SIZES)
    k4 = pick[7]
    eye, tgt, up = synth.random_poses(1, seed=62)[0]
    reqs[k4] = Request(7, synth.mvp(eye, tgt, up, 3840, 2160), 3840, 2160, pcr.HQ)
    budget = 2 << 30
    be = GpuBackend(dev, budget_bytes=budget, capacity=16)
    srv = Server(be, budget_bytes=budget)      # the measured server: the backend's default policy
    rng = np.random.default_rng(63)
    t1 = time.perf_counter()
    # a burst (queued before the loop starts, so that batches form), then
    # Poisson arrivals at about 1,500 requests/s while earlier batches run
    futs = [srv.submit(r) for r in reqs[:80]]
    srv.start()
    for r, gap in zip(reqs[80:], rng.exponential(1.0 / 1500.0, len(reqs) - 80)):
        time.sleep(gap)
        futs.append(srv.submit(r))
    res = [f.result(timeout=600) for f in futs]
    srv.stop()
    torch.cuda.synchronize()
    log(f"{len(res)} requests served in {time.perf_counter() - t1:.1f} s, batch sizes up to "
        f"{max(o.batch_size for o in res)}, mean {np.mean([o.batch_size for o in res]):.2f}")
    assert all(o.status == "ok" for o in res), [(o.rid, o.status, o.error) for o in res if o.status != "ok"][:5]
    assert max(o.batch_size for o in res) > 1
    assert srv.arena.used == 0
    # every result against the same request rendered alone (compared on the device)
    fb = torch.empty(pcr.fb_bytes(3840, 2160, pcr.HQ) // 8 + 1, dtype=torch.int64, device="cuda")
    alone = torch.empty(3840 * 2160, dtype=torch.int32, device="cuda")
    bad = []
    for r, o in zip(reqs, res):
        v = pcr.DEDUP if r.variant == pcr.BASIC else r.variant
        pcr.fb_clear(fb, r.w, r.h, v)
        pcr.render(dev[r.cloud], r.mvp, r.w, r.h, v, fb)
        pcr.resolve(fb, r.w, r.h, v, out=alone)
        if not torch.equal(o.image, alone[: r.w * r.h]):
            bad.append((r.rid, r.cloud, r.w, r.h, r.variant, o.batch_size))
    assert not bad, f"served images differ from solo renders: {bad[:10]}"
    log("every served image equals its solo render")
    for c, k in sorted(pick.items()):
        r, o = reqs[k], res[k]
        if r.variant == pcr.HQ:
            _, RG, BA = orc.render_hq(host[c], r.mvp, r.w, r.h)
            ref = orc.resolve_hq(RG, BA, r.w, r.h)
        else:
            ref = orc.resolve_basic(orc.render_basic(host[c], r.mvp, r.w, r.h), r.w, r.h)
        got = o.image.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref), (c, r.w, r.h, r.variant)
        assert got.any()
        log(f"cloud {c} ({SIZES[c]} points) {r.w}x{r.h} {'HQ' if r.variant == pcr.HQ else 'basic'}: equals the oracle")
    be.close()
