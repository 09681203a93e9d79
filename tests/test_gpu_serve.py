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


def test_results_equal_solo_under_load(orc, clouds):
    import torch
    host, dev = clouds
    be = GpuBackend(dev, budget_bytes=8 << 20, capacity=6)
    srv = Server(be, budget_bytes=8 << 20)
    srv.start()
    reqs = mixed_requests(60, seed=21)
    futs = []
    for r in reqs:
        futs.append(srv.submit(r))
        time.sleep(0.0002)
    res = [f.result(timeout=60) for f in futs]
    srv.stop()
    torch.cuda.synchronize()
    assert max(r.batch_size for r in res) > 1, "no batching happened"
    for r, out in zip(reqs, res):
        assert out.status == "ok"
        _, alone = render_frame(dev[r.cloud], r.mvp, r.w, r.h, r.variant)
        assert np.array_equal(out.image.cpu().numpy().view(np.uint32), alone), r
    for r, out in list(zip(reqs, res))[:8]:
        _, eimg = oracle_frame(orc, host[r.cloud], r.mvp, r.w, r.h, r.variant)
        assert np.array_equal(out.image.cpu().numpy().view(np.uint32), eimg)
    assert srv.arena.used == 0
    be.close()
