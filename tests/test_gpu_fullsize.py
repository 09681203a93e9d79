"""Parity at the measured workloads' full sizes, in the launch configuration the
benchmark times: whole frames bit-exact against the CPU oracle.

The oracle always renders the generator's own output.  Reordered clouds come
from the GPU reorder and must give the same image as the original order (the
image is a per-pixel min / sum, independent of order); the permutations
themselves are compared with the oracle's.
"""
import numpy as np
import pytest

from gpu_util import assert_same_fb, download_points, read_fb, upload
from paper_2104_07526_amd import pcr, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def log(msg):
    print(f"[fullsize] {msg}", flush=True)


def frame(d, m, W, H, variant, fb):
    import torch
    pcr.fb_clear(fb, W, H, variant)
    pcr.render(d, m, W, H, variant, fb)
    img = pcr.resolve(fb, W, H, variant)
    torch.cuda.synchronize()
    return img.cpu().numpy().view(np.uint32)


def test_terrain_100m_three_orders(orc):
    """100M terrain points, 1920x1080 oblique: basic and dedup on scanline,
    Morton and shuffled-Morton orders."""
    import torch
    n, W, H = 100_000_000, 1920, 1080
    pts = synth.terrain(n, seed=2)
    m = synth.terrain_oblique(W, H)
    ref = orc.render_basic(pts, m, W, H)
    ref_img = orc.resolve_basic(ref, W, H)
    log("terrain 100M: oracle frame done")
    d = upload(pts)
    clouds = {"scanline": d}
    mort, perm_m = pcr.reorder(d, pcr.ORDER_MORTON, 128, 3)
    msh, perm_s = pcr.reorder(d, pcr.ORDER_MORTON_SHUFFLE, 128, 3)
    torch.cuda.synchronize()
    clouds["morton"], clouds["morton_shuffle128"] = mort, msh
    # Both permutations equal the oracle's (stable sorts, same batch shuffle),
    # and the reordered clouds are the input gathered through them.
    for order, perm, cloud in ((0, perm_m, mort), (1, perm_s, msh)):
        got = perm.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, orc.reorder(pts, order, 128, 3)), order
        assert np.array_equal(download_points(cloud), pts[got]), order
        log(f"terrain 100M: order {order} permutation and gather match")
    del perm_m, perm_s, got
    for order, cloud in clouds.items():
        for variant in (pcr.BASIC, pcr.DEDUP):
            fb = pcr.alloc_fb(W, H, variant)
            img = frame(cloud, m, W, H, variant, fb)
            assert_same_fb(read_fb(fb, W, H, variant), ref, variant)
            assert np.array_equal(img, ref_img), (order, variant)
            log(f"terrain 100M: {order} variant {variant} bit-exact")


def test_buildings_300m_hq_1440p(orc):
    """300M building points, shuffled Morton, HQ at 2560x1440: depth, sums and
    image bit-exact."""
    import torch
    n, W, H = 300_000_000, 2560, 1440
    pts = synth.buildings(n, seed=4)
    m = synth.buildings_overview(W, H, seed=4)
    D, RG, BA = orc.render_hq(pts, m, W, H)
    ref_img = orc.resolve_hq(RG, BA, W, H)
    log("buildings 300M: oracle HQ frame done")
    d = upload(pts)
    del pts
    msh, _ = pcr.reorder(d, pcr.ORDER_MORTON_SHUFFLE, 128, 3, want_perm=False)
    del d
    torch.cuda.synchronize()
    fb = pcr.alloc_fb(W, H, pcr.HQ)
    img = frame(msh, m, W, H, pcr.HQ, fb)
    assert_same_fb(read_fb(fb, W, H, pcr.HQ), (D, RG, BA), pcr.HQ)
    assert np.array_equal(img, ref_img)
    cnt = (BA & 0xFFFFFFFF).astype(np.int64)
    assert cnt.max() < 16_843_009          # per-channel sums are exact averages
    assert (cnt > 1).sum() > 100_000       # blending actually happens
    assert (cnt > 255).sum() > 1000        # the robust form's fast words overflow somewhere
    log("buildings 300M: HQ bit-exact")
    # the robust single-atomic form (fast word + fallback words) on the same frame
    from test_gpu_hq_robust import assert_valid_fast_words, read_robust
    RB = pcr.HQ | pcr.F_HQ_ROBUST
    fb = pcr.alloc_fb(W, H, RB)
    img = frame(msh, m, W, H, RB, fb)
    gD, gRG, gBA, F = read_robust(fb, W, H)
    assert np.array_equal(gD, D) and np.array_equal(gRG, RG) and np.array_equal(gBA, BA)
    assert_valid_fast_words(F)
    assert np.array_equal(img, ref_img)
    log("buildings 300M: robust HQ bit-exact")


def test_buildings_796m_1080p(orc):
    """The 796M-point (12.7 GB) cloud, shuffled Morton, 1920x1080: dedup, basic
    and HQ frames bit-exact."""
    import torch
    n, W, H = 796_000_000, 1920, 1080
    pts = synth.buildings(n, seed=4)
    m = synth.buildings_overview(W, H, seed=4)
    log("buildings 796M: generated")
    ref = orc.render_basic(pts, m, W, H)
    log("buildings 796M: oracle basic frame done")
    D, RG, BA = orc.render_hq(pts, m, W, H)
    log("buildings 796M: oracle HQ frame done")
    d = upload(pts)
    del pts
    msh, _ = pcr.reorder(d, pcr.ORDER_MORTON_SHUFFLE, 128, 3, want_perm=False)
    del d
    torch.cuda.synchronize()
    for variant in (pcr.DEDUP, pcr.BASIC):
        fb = pcr.alloc_fb(W, H, variant)
        frame(msh, m, W, H, variant, fb)
        assert_same_fb(read_fb(fb, W, H, variant), ref, variant)
        log(f"buildings 796M: variant {variant} bit-exact")
    fb = pcr.alloc_fb(W, H, pcr.HQ)
    frame(msh, m, W, H, pcr.HQ, fb)
    assert_same_fb(read_fb(fb, W, H, pcr.HQ), (D, RG, BA), pcr.HQ)


def test_batch_145m_64_views(orc):
    """The batched workload: 145M points (terrain + buildings), 64 views at
    720p / 1080p / 4K, basic and HQ.  Under every launch shape the autotuner
    may pick, two replays of the plan give each view's single-view image; one
    view per resolution equals the oracle."""
    import torch
    from paper_2104_07526_amd import tune
    nt, nb = 100_000_000, 45_000_000
    pts = synth.terrain_and_buildings(nt, nb, seed=5)
    d = upload(pts)
    msh, _ = pcr.reorder(d, pcr.ORDER_MORTON_SHUFFLE, 128, 3, want_perm=False)
    del d
    res = [(1280, 720), (1920, 1080), (3840, 2160)]
    views, pviews, fbs, imgs, alone = [], [], [], [], []
    for i, (eye, tgt, up) in enumerate(synth.random_poses(64, seed=5)):
        W, H = res[i % 3]
        var = pcr.BASIC if i % 2 == 0 else pcr.HQ
        m = synth.mvp(eye, tgt, up, W, H)
        fb = pcr.alloc_fb(W, H, var)
        alone.append(frame(msh, m, W, H, var, fb))
        im = torch.empty(W * H, dtype=torch.int32, device="cuda")
        views.append((m, W, H, var))
        fbs.append(fb)        # the views hold raw pointers: keep every buffer alive
        imgs.append(im)
        pviews.append(pcr.make_view(m, W, H, var, fb, im))
    for k in (0, 1, 5):        # 720p basic, 1080p HQ, 4K HQ
        m, W, H, var = views[k]
        if var == pcr.HQ:
            _, RG, BA = orc.render_hq(pts, m, W, H)
            ref = orc.resolve_hq(RG, BA, W, H)
        else:
            ref = orc.resolve_basic(orc.render_basic(pts, m, W, H), W, H)
        assert np.array_equal(alone[k], ref), k
        log(f"batch 145M: view {k} single-view render equals the oracle")
    for t in [None] + tune.BATCH_CANDIDATES:
        plan = pcr.BatchPlan(msh, 64, tune=t)
        for rep in range(2):
            for im in imgs:
                im.fill_(0)
            plan.launch(pviews)
            torch.cuda.synchronize()
            for k, im in enumerate(imgs):
                assert np.array_equal(im.cpu().numpy().view(np.uint32), alone[k]), (t, rep, k)
        log(f"batch 145M: plan {t} matches single-view renders on two replays")
        plan.close()
