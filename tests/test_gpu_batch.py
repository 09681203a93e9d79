"""Batched multi-view plans (one hipGraph replay per launch): every view equals
the oracle's render of that view alone and the single-view GPU render, on
repeated replays with eager work in between."""
import numpy as np
import pytest

from gpu_util import assert_same_fb, oracle_frame, read_fb, render_frame, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu

SIZES = [(96, 54), (160, 90), (64, 64), (200, 120)]


def make_views(k, seed, variants=(pcr.BASIC, pcr.DEDUP, pcr.HQ)):
    poses = synth.random_poses(k, seed=seed)
    out = []
    for i, (eye, tgt, up) in enumerate(poses):
        W, H = SIZES[i % len(SIZES)]
        out.append((synth.mvp(eye, tgt, up, W, H), W, H, variants[i % len(variants)]))
    return out


def run_batch(plan, views):
    import torch
    bufs, pv = [], []
    for m, W, H, var in views:
        fb = pcr.alloc_fb(W, H, var)
        img = torch.empty(W * H, dtype=torch.int32, device="cuda")
        bufs.append((fb, img))
        pv.append(pcr.make_view(m, W, H, var, fb, img))
    plan.launch(pv)
    torch.cuda.synchronize()
    return bufs


@pytest.fixture(scope="module")
def scene():
    pts = synth.terrain_and_buildings(300_000, 100_000, seed=5)
    return pts, upload(pts)


@pytest.mark.parametrize("tune", [None, {"ppt": 4}, {"ppt": 8, "group": 2}, {"ppt": 16, "slots": 256},
                                  {"ppt": 8, "group": 1}, {"ppt": 2, "group": 1, "slots": 256},
                                  {"ppt": 8, "group": 4, "wg": 64}, {"ppt": 4, "group": 16, "wg": 128}])
def test_views_match_oracle(orc, scene, tune):
    pts, d = scene
    views = make_views(9, seed=11)
    plan = pcr.BatchPlan(d, capacity=12, tune=tune)
    bufs = run_batch(plan, views)
    for (m, W, H, var), (fb, img) in zip(views, bufs):
        efb, eimg = oracle_frame(orc, pts, m, W, H, var)
        assert_same_fb(read_fb(fb, W, H, var), efb, var)
        assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg)
    plan.close()


@pytest.mark.parametrize("tune", [None, {"group": 1}])
def test_replays_with_eager_work_between(orc, scene, tune):
    """The graph is replayed with new views each time; eager single-view
    renders run between the replays; every replay is checked."""
    pts, d = scene
    plan = pcr.BatchPlan(d, capacity=6, tune=tune)
    for rep in range(4):
        views = make_views(5 + rep % 2, seed=100 + rep)
        bufs = run_batch(plan, views)
        m0, W0, H0, v0 = views[0]
        _, eager = render_frame(d, m0, W0, H0, v0)
        for (m, W, H, var), (fb, img) in zip(views, bufs):
            _, eimg = oracle_frame(orc, pts, m, W, H, var)
            assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg), (rep, var)
        assert np.array_equal(bufs[0][1].cpu().numpy().view(np.uint32), eager)
    plan.close()


def test_empty_unused_and_capacity(orc, scene):
    import torch
    pts, d = scene
    plan = pcr.BatchPlan(d, capacity=3)
    plan.launch([])
    torch.cuda.synchronize()
    views = make_views(2, seed=3)
    bufs, fbs = [], []
    pv = []
    for m, W, H, var in views:
        fb = pcr.alloc_fb(W, H, var)
        img = torch.zeros(W * H, dtype=torch.int32, device="cuda")
        bufs.append(img)
        fbs.append(fb)          # the views hold raw pointers: keep the buffers alive
        pv.append(pcr.make_view(m, W, H, var, fb, img))
    pv[1].variant = -1          # unused slot: left untouched
    plan.launch(pv)
    torch.cuda.synchronize()
    m, W, H, var = views[0]
    _, eimg = oracle_frame(orc, pts, m, W, H, var)
    assert np.array_equal(bufs[0].cpu().numpy().view(np.uint32), eimg)
    assert not bufs[1].cpu().numpy().any()
    with pytest.raises(pcr.PcrError) as e:
        plan.launch(pv * 2)
    assert e.value.code == pcr.EINVAL
    plan.close()


def test_large_views_group_split(orc):
    """Views whose framebuffers exceed one group's 2 GiB are split over
    several point passes: three 8K HQ views (663 MB each) and an 8K basic
    view (265 MB) pass the limit at the fourth HQ view; plus 1080p and 720p
    views, over a 2M-point terrain."""
    import torch
    pts = synth.terrain(2_000_000, seed=2)
    d = upload(pts)
    W8, H8 = 7680, 4320
    views = [(synth.terrain_oblique(W8, H8), W8, H8, pcr.HQ),
             (synth.terrain_overview(W8, H8), W8, H8, pcr.HQ),
             (synth.terrain_closeup(W8, H8), W8, H8, pcr.BASIC),
             (synth.terrain_oblique(1920, 1080), 1920, 1080, pcr.DEDUP),
             (synth.terrain_closeup(W8, H8), W8, H8, pcr.HQ),
             (synth.terrain_overview(1280, 720), 1280, 720, pcr.HQ)]
    fbb = [pcr.fb_bytes(W, H, var) for _, W, H, var in views]
    assert sum(fbb[:4]) <= 2 << 30 < sum(fbb[:5])
    plan = pcr.BatchPlan(d, capacity=6)
    bufs = run_batch(plan, views)
    for (m, W, H, var), (fb, img) in zip(views, bufs):
        _, eimg = oracle_frame(orc, pts, m, W, H, var)
        assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg)
    plan.close()
    torch.cuda.synchronize()


def test_many_views_fill_the_shared_table(orc):
    """Sixteen views per group over a dense terrain with small tables (256 LDS
    slots): the shared (view, pixel) table fills past half during a tile and
    is flushed between views many times; every view still equals the oracle."""
    import torch
    pts = synth.terrain(1_500_000, seed=2)
    d = upload(pts)
    views = []
    for i, (eye, tgt, up) in enumerate(synth.random_poses(16, seed=77)):
        W, H = [(320, 180), (256, 256)][i % 2]
        views.append((synth.mvp(eye, tgt, up, W, H), W, H, [pcr.BASIC, pcr.HQ][i % 2]))
    for tune in ({"ppt": 4, "group": 16, "slots": 256}, {"ppt": 8, "group": 16, "slots": 256},
                 {"ppt": 8, "group": 16, "wg": 64}):
        plan = pcr.BatchPlan(d, capacity=16, tune=tune)
        for _ in range(2):
            bufs = run_batch(plan, views)
            for (m, W, H, var), (fb, img) in zip(views, bufs):
                _, eimg = oracle_frame(orc, pts, m, W, H, var)
                assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg)
        plan.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("tune", [None, {"group": 1}])
def test_back_to_back_launches_of_varying_size(orc, scene, tune):
    """Launches of 8, 2, 5, 1 and 8 views enqueued back to back on one stream
    without waiting (per-view plans enable only the slots each launch uses);
    every image of every launch equals the oracle."""
    import torch
    pts, d = scene
    plan = pcr.BatchPlan(d, capacity=8, tune=tune)
    launches = []
    for k, cnt in enumerate((8, 2, 5, 1, 8)):
        views = make_views(cnt, seed=300 + k)
        bufs, pv = [], []
        for m, W, H, var in views:
            fb = pcr.alloc_fb(W, H, var)
            img = torch.zeros(W * H, dtype=torch.int32, device="cuda")
            bufs.append((fb, img))
            pv.append(pcr.make_view(m, W, H, var, fb, img))
        plan.launch(pv)
        launches.append((views, bufs))
    torch.cuda.synchronize()
    for k, (views, bufs) in enumerate(launches):
        for (m, W, H, var), (fb, img) in zip(views, bufs):
            _, eimg = oracle_frame(orc, pts, m, W, H, var)
            assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg), (k, var)
    plan.close()


def test_one_call_batches_over_cached_plans(orc, scene):
    """pcr_render_batch: view sets of 3 and 7 (two cached plans), and the same
    plan launched on two streams back to back without waiting; every image
    equals the oracle."""
    import torch
    pts, d = scene
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    runs = []
    for k, (cnt, stream) in enumerate(((3, None), (7, None), (3, s1), (3, s2), (7, s1))):
        views = make_views(cnt, seed=500 + k)
        bufs, pv = [], []
        for m, W, H, var in views:
            fb = pcr.alloc_fb(W, H, var)
            img = torch.zeros(W * H, dtype=torch.int32, device="cuda")
            bufs.append((fb, img))
            pv.append(pcr.make_view(m, W, H, var, fb, img))
        if stream is not None:
            stream.wait_stream(torch.cuda.current_stream())   # the zeroed images
        pcr.render_batch(d, pv, stream=stream)
        runs.append((views, bufs))
    torch.cuda.synchronize()
    for k, (views, bufs) in enumerate(runs):
        for (m, W, H, var), (fb, img) in zip(views, bufs):
            _, eimg = oracle_frame(orc, pts, m, W, H, var)
            assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg), (k, var)
    pcr.release_batch_plans()


def test_destroy_and_eviction_wait_for_launches_in_flight(orc, scene):
    """A plan closed right after its launch, and cached plans evicted (ten
    launch shapes through a cache of eight) while their launches may still
    run: every image equals the single-view render, three of them the
    oracle."""
    import torch
    pts, d = scene
    torch.cuda.synchronize()
    runs = []
    plan = pcr.BatchPlan(d, capacity=4)
    views = make_views(3, seed=700)
    bufs, pv = [], []
    for m, W, H, var in views:
        fb = pcr.alloc_fb(W, H, var)
        img = torch.zeros(W * H, dtype=torch.int32, device="cuda")
        bufs.append((fb, img))
        pv.append(pcr.make_view(m, W, H, var, fb, img))
    plan.launch(pv)
    plan.close()
    runs.append((views, bufs))
    from paper_2104_07526_amd.tune import BATCH_CANDIDATES
    tunes = BATCH_CANDIDATES[::2][:10]             # per-view and batched shapes
    for k, t in enumerate(tunes):
        views = make_views(3, seed=710 + k)
        bufs, pv = [], []
        for m, W, H, var in views:
            fb = pcr.alloc_fb(W, H, var)
            img = torch.zeros(W * H, dtype=torch.int32, device="cuda")
            bufs.append((fb, img))
            pv.append(pcr.make_view(m, W, H, var, fb, img))
        pcr.render_batch(d, pv, tune=t)
        runs.append((views, bufs))
    torch.cuda.synchronize()
    for k, (views, bufs) in enumerate(runs):
        for (m, W, H, var), (fb, img) in zip(views, bufs):
            _, alone = render_frame(d, m, W, H, var)
            assert np.array_equal(img.cpu().numpy().view(np.uint32), alone), (k, var)
    for (m, W, H, var), (_, img) in zip(*runs[0]):
        _, eimg = oracle_frame(orc, pts, m, W, H, var)
        assert np.array_equal(img.cpu().numpy().view(np.uint32), eimg)
    pcr.release_batch_plans()
