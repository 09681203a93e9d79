"""The render server on the GPU: every result of a mixed, overlapping request
load equals the same request rendered alone (tolerance 0)."""
import time

import numpy as np
import pytest

from gpu_util import oracle_frame, render_frame, upload
from paper_2104_07526_amd import pcr, synth
from paper_2104_07526_amd.serve import GpuBackend, Request, Server

pytestmark = pytest.mark.gpu

RES = [(160, 90), (96, 96), (320, 180), (64, 48)]


@pytest.fixture(scope="module")
def clouds():
    host = [synth.terrain(400_000, seed=2), synth.buildings(300_000, seed=4),
            synth.terrain_and_buildings(200_000, 100_000, seed=5)]
    return host, [upload(h) for h in host]


def mixed_requests(k, seed):
    rng = np.random.default_rng(seed)
    poses = synth.random_poses(k, seed=seed)
    out = []
    for i, (eye, tgt, up) in enumerate(poses):
        w, h = RES[int(rng.integers(0, len(RES)))]
        v = [pcr.BASIC, pcr.DEDUP, pcr.HQ][int(rng.integers(0, 3))]
        out.append(Request(int(rng.integers(0, 3)), synth.mvp(eye, tgt, up, w, h), w, h, v))
    return out


@pytest.mark.parametrize("streams,max_points,big,beside", [(8, None, None, None), (2, 700_000, None, None),
                                                           (16, None, None, None), (8, 700_000, 500_000, None),
                                                           (8, 700_000, 500_000, 1)])
def test_results_equal_solo_under_load(orc, clouds, streams, max_points, big, beside):
    """A burst (every request admitted before the loop runs, so batches hold
    several views) followed by a trickle served by the threaded loop while
    earlier batches are still on the device; with several stream pools,
    batches capped by points, large batches run one at a time, and few small
    batches beside a large one."""
    import torch
    host, dev = clouds
    be = GpuBackend(dev, budget_bytes=8 << 20, capacity=6, streams=streams)
    srv = Server(be, budget_bytes=8 << 20, max_batch_points=max_points, big_points=big, small_beside_big=beside)
    burst = mixed_requests(24, seed=21)
    futs = [srv.submit(r) for r in burst]
    srv.drain()
    sizes = [f.result().batch_size for f in futs]
    assert max(sizes) > 1, f"no batching in the burst: {sizes}"
    trickle = mixed_requests(40, seed=22)
    srv.start()
    for r in trickle:
        futs.append(srv.submit(r))
        time.sleep(0.0002)
    res = [f.result(timeout=60) for f in futs]
    srv.stop()
    torch.cuda.synchronize()
    reqs = burst + trickle
    bad = []
    for r, out in zip(reqs, res):
        assert out.status == "ok", (out.status, out.error)
        _, alone = render_frame(dev[r.cloud], r.mvp, r.w, r.h, r.variant)
        got = out.image.cpu().numpy().view(np.uint32)
        if not np.array_equal(got, alone):
            bad.append((r.rid, r.cloud, r.w, r.h, r.variant, out.batch_size, int((got != alone).sum())))
    assert not bad, f"served images differ from solo renders: {bad[:10]}"
    for r, out in list(zip(reqs, res))[:8]:
        _, eimg = oracle_frame(orc, host[r.cloud], r.mvp, r.w, r.h, r.variant)
        assert np.array_equal(out.image.cpu().numpy().view(np.uint32), eimg), r.rid
    assert srv.arena.used == 0, srv.arena.used
    be.close()


def test_requests_no_plan_can_render_are_refused_alone(clouds):
    """A packed-HQ view, an unknown variant, a view past 2^27 - 1 pixels and a
    short matrix are refused at submit; the valid requests submitted around
    them are batched together and equal their solo renders."""
    import torch
    _, dev = clouds
    be = GpuBackend(dev, budget_bytes=8 << 20, capacity=6)
    srv = Server(be, budget_bytes=8 << 20)
    good = [r for r in mixed_requests(12, seed=31) if r.cloud == 0][:3]
    assert len(good) == 3
    m = good[0].mvp
    bad = [Request(0, m, 64, 48, pcr.HQ | pcr.F_HQ_PACKED), Request(0, m, 64, 48, 7),
           Request(0, m, 16384, 8192, pcr.BASIC), Request(0, m[:12], 64, 48, pcr.BASIC)]
    futs = [srv.submit(r) for r in (good[0], bad[0], good[1], bad[1], bad[2], good[2], bad[3])]
    for i in (1, 3, 4, 6):
        assert futs[i].done() and futs[i].result().status == "rejected", i
    srv.drain()
    torch.cuda.synchronize()
    for f, r in zip((futs[0], futs[2], futs[5]), good):
        out = f.result()
        assert out.status == "ok", (out.status, out.error)
        assert out.batch_size == 3
        _, alone = render_frame(dev[r.cloud], r.mvp, r.w, r.h, r.variant)
        assert np.array_equal(out.image.cpu().numpy().view(np.uint32), alone)
    assert srv.rejected == 4 and srv.arena.used == 0
    be.close()
