"""The serving scheduler on the CPU, with a test backend that renders through
the CPU oracle and completes batches after a simulated delay: admission by
framebuffer memory, arrival order, continuous batching, failures, cancellation,
and results equal to solo renders."""
import time

import numpy as np
import pytest

from paper_2104_07526_amd import pcr, synth
from paper_2104_07526_amd.serve import Arena, Request, Server, percentile


class OracleBackend:
    """Test backend: batches are rendered by the CPU oracle at launch and
    reported complete `delay` seconds later."""

    def __init__(self, orc, clouds, capacity=4, slots=2, delay=0.002, fail_variant=None, streams=None):
        self.orc = orc
        self.clouds = clouds
        self.capacity = capacity
        self.points = [len(c) for c in clouds]
        self.delay = delay
        self.fail_variant = fail_variant
        self.busy = [[None] * slots for _ in clouds]
        self.streams = streams       # batches in flight at once over all clouds (None: no limit)
        self.batches = []
        self.launched = []           # (cloud, [rid, ...]) in launch order

    def bytes_for(self, req):
        return (pcr.fb_bytes(req.w, req.h, req.variant) + 255) // 256 * 256

    def new_image(self, req):
        return np.zeros(req.w * req.h, np.uint32)

    def free_slot(self, cloud):
        if self.streams is not None and sum(b is not None for row in self.busy for b in row) >= self.streams:
            return None
        for i, b in enumerate(self.busy[cloud]):
            if b is None:
                return i
        return None

    def launch(self, cloud, slot, reqs, offsets, images):
        if self.fail_variant is not None and any(r.variant == self.fail_variant for r in reqs):
            raise RuntimeError("injected launch failure")
        for r, img in zip(reqs, images):
            img[:] = solo(self.orc, self.clouds[cloud], r)
        self.busy[cloud][slot] = time.perf_counter() + self.delay
        self.batches.append(len(reqs))
        self.launched.append((cloud, [r.rid for r in reqs]))
        return (cloud, slot)

    def done(self, h):
        t = self.busy[h[0]][h[1]]
        return t is None or time.perf_counter() >= t

    def retire(self, h):
        self.busy[h[0]][h[1]] = None


def solo(orc, pts, r):
    if r.variant == pcr.HQ:
        _, RG, BA = orc.render_hq(pts, r.mvp, r.w, r.h)
        return orc.resolve_hq(RG, BA, r.w, r.h)
    return orc.resolve_basic(orc.render_basic(pts, r.mvp, r.w, r.h), r.w, r.h)


@pytest.fixture(scope="module")
def clouds():
    return [synth.terrain(20_000, seed=2), synth.buildings(15_000, seed=4)]


def requests(k, seed=0, sizes=((32, 18), (64, 36), (48, 48))):
    rng = np.random.default_rng(seed)
    poses = synth.random_poses(k, seed=seed)
    out = []
    for i, (eye, tgt, up) in enumerate(poses):
        w, h = sizes[i % len(sizes)]
        v = pcr.HQ if rng.random() < 0.3 else pcr.BASIC
        out.append(Request(int(rng.integers(0, 2)), synth.mvp(eye, tgt, up, w, h), w, h, v))
    return out


def test_arena_first_fit_and_coalescing():
    a = Arena(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(2000) is None
    a.release(y, 1000)
    assert a.alloc(2000) is None          # hole of 1024 only
    a.release(x, 1000)
    assert a.alloc(2000) == 0             # coalesced with the previous hole
    a.release(0, 2000)
    a.release(z, 1000)
    assert a.free == [(0, 4096)] and a.used == 0


def test_all_results_equal_solo_renders(orc, clouds):
    be = OracleBackend(orc, clouds)
    srv = Server(be, budget_bytes=1 << 24)
    reqs = requests(24, seed=1)
    futs = [srv.submit(r) for r in reqs]
    srv.drain()
    for r, f in zip(reqs, futs):
        res = f.result()
        assert res.status == "ok"
        assert np.array_equal(res.image, solo(orc, clouds[r.cloud], r))
    assert srv.arena.used == 0 and srv.completed == len(reqs)


def test_admission_waits_for_memory_in_arrival_order(orc, clouds):
    """A budget that holds about two framebuffers: requests wait (none is
    dropped), memory in use never exceeds the budget, admission follows
    arrival order."""
    be = OracleBackend(orc, clouds, delay=0.003)
    one = be.bytes_for(Request(0, None, 64, 36, pcr.HQ))
    srv = Server(be, budget_bytes=2 * one)
    reqs = [Request(i % 2, synth.terrain_oblique(64, 36), 64, 36, pcr.HQ) for i in range(10)]
    futs = [srv.submit(r) for r in reqs]
    peak = 0
    order = []
    while srv.step():
        peak = max(peak, srv.arena.used)
        for items in srv.admitted.values():
            order += [t[0].rid for t in items if t[0].rid not in order]
        for item in srv.inflight:
            order += [t[0].rid for t in item[1] if t[0].rid not in order]
        time.sleep(1e-4)
    assert peak <= 2 * one
    assert order == sorted(order)
    assert all(f.result().status == "ok" for f in futs)


def test_continuous_batching_groups_arrivals(orc, clouds):
    """Requests that arrive while a batch is on the device join the next batch
    of their cloud."""
    be = OracleBackend(orc, clouds, capacity=8, slots=1, delay=0.02)
    srv = Server(be, budget_bytes=1 << 26)
    srv.submit(requests(1, seed=3)[0])
    srv.step()                               # first batch launched alone
    more = [Request(0, synth.terrain_oblique(32, 18), 32, 18, pcr.BASIC) for _ in range(6)]
    futs = [srv.submit(r) for r in more]
    srv.drain()
    assert max(be.batches) >= 5
    assert all(f.result().batch_size >= 5 for f in futs)


def test_oversized_request_is_rejected(orc, clouds):
    be = OracleBackend(orc, clouds)
    srv = Server(be, budget_bytes=4096)
    f = srv.submit(Request(0, synth.terrain_oblique(64, 64), 64, 64, pcr.BASIC))
    assert f.result().status == "rejected"
    f = srv.submit(Request(5, synth.terrain_oblique(8, 8), 8, 8, pcr.BASIC))
    assert f.result().status == "rejected"
    assert not srv.step()


def test_request_the_backend_cannot_render_is_rejected_alone(orc, clouds):
    """bytes_for raising refuses that request at submit; the requests around
    it are batched and served."""
    class Picky(OracleBackend):
        def bytes_for(self, req):
            if req.variant == pcr.HQ:
                raise ValueError("no HQ here")
            return super().bytes_for(req)

    be = Picky(orc, clouds, capacity=4)
    srv = Server(be, budget_bytes=1 << 24)
    reqs = [Request(0, synth.terrain_oblique(32, 18), 32, 18, v) for v in (pcr.BASIC, pcr.HQ, pcr.BASIC)]
    futs = [srv.submit(r) for r in reqs]
    assert futs[1].done() and futs[1].result().status == "rejected"
    assert "no HQ here" in futs[1].result().error
    srv.drain()
    assert [futs[0].result().status, futs[2].result().status] == ["ok", "ok"]
    assert futs[0].result().batch_size == 2
    assert srv.rejected == 1 and srv.arena.used == 0


def test_launch_failure_fails_its_batch_and_server_continues(orc, clouds):
    be = OracleBackend(orc, clouds, capacity=1, fail_variant=pcr.HQ)
    srv = Server(be, budget_bytes=1 << 24)
    reqs = [Request(0, synth.terrain_oblique(32, 18), 32, 18, v) for v in (pcr.BASIC, pcr.HQ, pcr.BASIC)]
    futs = [srv.submit(r) for r in reqs]
    srv.drain()
    st = [f.result().status for f in futs]
    assert st == ["ok", "error", "ok"]
    assert "injected" in futs[1].result().error
    assert srv.arena.used == 0


def test_cancelled_requests_are_skipped(orc, clouds):
    be = OracleBackend(orc, clouds)
    srv = Server(be, budget_bytes=1 << 24)
    f1 = srv.submit(requests(1, seed=5)[0])
    f2 = srv.submit(requests(1, seed=6)[0])
    assert f2.cancel()
    srv.drain()
    assert f1.result().status == "ok" and f2.cancelled()
    assert sum(be.batches) == 1


def test_threaded_loop_and_latency_stats(orc, clouds):
    be = OracleBackend(orc, clouds, delay=0.001)
    srv = Server(be, budget_bytes=1 << 24)
    srv.start()
    futs = []
    for r in requests(12, seed=7):
        futs.append(srv.submit(r))
        time.sleep(0.001)
    res = [f.result(timeout=30) for f in futs]
    srv.stop()
    lat = [r.latency for r in res]
    assert all(x > 0 for x in lat)
    assert percentile(lat, 50) <= percentile(lat, 99)


def test_oldest_request_launches_first_across_clouds(orc, clouds):
    """With one batch in flight at a time, batches start in the order of their
    oldest request, whatever the cloud."""
    be = OracleBackend(orc, clouds, capacity=8, streams=1, delay=0.01)
    srv = Server(be, budget_bytes=1 << 26)
    m = synth.terrain_oblique(32, 18)
    first = srv.submit(Request(0, m, 32, 18, pcr.BASIC))
    srv.step()                               # on the device
    later = [srv.submit(Request(c, m, 32, 18, pcr.BASIC)) for c in (1, 0, 1, 0, 0)]
    srv.drain()
    heads = [min(rids) for _, rids in be.launched]
    assert heads == sorted(heads)
    assert [c for c, _ in be.launched] == [0, 1, 0]
    assert all(f.result().status == "ok" for f in [first] + later)


def test_batch_points_cap(orc, clouds):
    """max_batch_points bounds the views of one batch by the cloud's size (at
    least one view), and images stay equal to solo renders."""
    be = OracleBackend(orc, clouds, capacity=8, slots=1, delay=0.01)
    cap = 2 * len(clouds[0]) + 10
    srv = Server(be, budget_bytes=1 << 26, max_batch_points=cap)
    reqs = [Request(c, synth.terrain_oblique(32, 18), 32, 18, pcr.BASIC) for c in (0,) * 7 + (1,) * 7]
    futs = [srv.submit(r) for r in reqs]
    srv.drain()
    per_cloud = {0: [], 1: []}
    for c, rids in be.launched:
        per_cloud[c].append(len(rids))
    assert max(per_cloud[0]) == 2 and max(per_cloud[1]) == min(8, cap // len(clouds[1]))
    for r, f in zip(reqs, futs):
        assert np.array_equal(f.result().image, solo(orc, clouds[r.cloud], r))
    srv2 = Server(OracleBackend(orc, clouds), budget_bytes=1 << 20, max_batch_points=1)
    assert srv2._batch_limit(0) == 1


def test_big_batches_run_one_at_a_time(orc, clouds):
    """With big_points, batches streaming at least that many points never
    overlap each other (an HQ view counts its cloud twice), while small
    batches run beside them; every image equals its solo render."""
    be = OracleBackend(orc, clouds, capacity=1, slots=3, delay=0.01)
    srv = Server(be, budget_bytes=1 << 26, big_points=len(clouds[0]) + 1)
    m = synth.terrain_oblique(32, 18)
    reqs = ([Request(0, m, 32, 18, pcr.HQ) for _ in range(3)] + [Request(1, m, 32, 18, pcr.BASIC) for _ in range(3)]
            + [Request(0, m, 32, 18, pcr.BASIC)])
    futs = [srv.submit(r) for r in reqs]
    most_big, most_small = 0, 0
    while srv.step():
        big = [it for it in srv.inflight if it[3]]
        most_big = max(most_big, len(big))
        most_small = max(most_small, len(srv.inflight) - len(big))
        time.sleep(2e-4)
    assert most_big == 1 and most_small >= 2
    for r, f in zip(reqs, futs):
        assert np.array_equal(f.result().image, solo(orc, clouds[r.cloud], r))


def test_small_batches_beside_a_big_one_are_capped(orc, clouds):
    """small_beside_big bounds the smaller batches in flight while a big one
    runs; without a big batch they are not limited."""
    be = OracleBackend(orc, clouds, capacity=1, slots=8, delay=0.01)
    srv = Server(be, budget_bytes=1 << 26, big_points=len(clouds[0]) + 1, small_beside_big=1)
    m = synth.terrain_oblique(32, 18)
    reqs = [Request(0, m, 32, 18, pcr.HQ)] + [Request(1, m, 32, 18, pcr.BASIC) for _ in range(6)]
    futs = [srv.submit(r) for r in reqs]
    most_small_with_big, most_small = 0, 0
    while srv.step():
        big = sum(1 for it in srv.inflight if it[3])
        small = len(srv.inflight) - big
        if big:
            most_small_with_big = max(most_small_with_big, small)
        most_small = max(most_small, small)
        time.sleep(2e-4)
    assert most_small_with_big == 1 and most_small > 1
    for r, f in zip(reqs, futs):
        assert np.array_equal(f.result().image, solo(orc, clouds[r.cloud], r))


def test_gpu_backend_refuses_what_no_batch_plan_renders():
    """GpuBackend.bytes_for (host only): the aligned framebuffer size of a
    valid request; PcrError for an unknown variant, the packed HQ flag, views
    of 2^27 or more pixels and a matrix without 16 floats."""
    from paper_2104_07526_amd.serve import GpuBackend
    be = GpuBackend.__new__(GpuBackend)          # no device state is needed for sizes
    m = synth.terrain_oblique(64, 48)
    assert be.bytes_for(Request(0, m, 64, 48, pcr.BASIC)) == 8 * 64 * 48
    assert be.bytes_for(Request(0, m, 100, 30, pcr.HQ)) % 256 == 0
    bad = [(Request(0, m, 64, 48, 7), pcr.EINVAL), (Request(0, m, 0, 48, pcr.BASIC), pcr.EINVAL),
           (Request(0, m, 64, 48, pcr.HQ | pcr.F_HQ_PACKED), pcr.EUNSUPPORTED),
           (Request(0, m, 16384, 8192, pcr.BASIC), pcr.EINVAL), (Request(0, m[:12], 64, 48, pcr.BASIC), pcr.EINVAL)]
    for req, code in bad:
        with pytest.raises(pcr.PcrError) as e:
            be.bytes_for(req)
        assert e.value.code == code, req
