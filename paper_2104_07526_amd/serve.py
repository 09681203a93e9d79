"""Continuous-batching render server over resident point clouds.

Requests (cloud, camera, resolution, variant) arrive at any time.  The
scheduler admits them in arrival order while their framebuffers fit the
framebuffer memory budget.  Whenever a batch slot is free it launches, oldest
waiting request first, one batched multi-view render of everything admitted
for that request's cloud so far.  A slot is a free batch plan of the cloud
(two per cloud, so a new batch of a cloud starts while its previous batch is
still on the GPU) and a free stream of a small pool: batches on different
streams overlap on the device.  Optionally, batches that stream many points
run one at a time beside any number of small ones, and the views of one batch
are capped by the cloud's size.  A request's image is the same as rendering it
alone (integer min / sum updates).

The scheduler is independent of the device: a backend supplies buffer sizes,
batch launches and completion queries.  ``GpuBackend`` drives libpcr batch
plans; tests drive the scheduler with their own backends.
"""
from __future__ import annotations

import bisect
import dataclasses
import threading
import time
from concurrent.futures import Future

import numpy as np

from . import pcr

ALIGN = 256


def _align(n: int) -> int:
    return (n + ALIGN - 1) // ALIGN * ALIGN


@dataclasses.dataclass
class Request:
    cloud: int
    mvp: np.ndarray
    w: int
    h: int
    variant: int
    arrival: float = 0.0            # time.perf_counter() seconds
    rid: int = -1


@dataclasses.dataclass
class Result:
    rid: int
    image: object                   # device tensor (GPU backend) or array
    arrival: float
    launched: float
    finished: float
    batch_size: int
    status: str = "ok"
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Arena:
    """First-fit allocator of byte ranges inside one preallocated region
    (framebuffer memory budget).  Host bookkeeping only."""

    def __init__(self, size: int):
        self.size = size
        self.free = [(0, size)]      # sorted (offset, length), coalesced
        self.used = 0

    def alloc(self, n: int):
        n = _align(max(n, 1))
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                self.used += n
                return off
        return None

    def release(self, off: int, n: int):
        n = _align(max(n, 1))
        self.used -= n
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, n))
        # coalesce with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)


class GpuBackend:
    """libpcr batch plans on a pool of torch streams.  Framebuffers are carved
    from one device arena (the admission budget); each request's image is its
    own device tensor, written directly by the batch's resolve.  The plans run
    in their default shape unless ``tune`` says otherwise: grouped passes, so
    the requests of one batch share one read of their cloud per group of views.
    At most ``streams`` batches are in flight, each on a stream of its own, and
    at most ``plans_per_cloud`` per cloud.  The defaults (two streams, one plan
    per cloud) let the requests of a cloud gather behind its running batch and
    share the next one's point stream: measured on the eight-cloud request
    load, they serve 16% more points per second than one-request-at-a-time
    service past saturation, where eight streams and two plans per cloud
    overlapped single requests and gained nothing."""

    def __init__(self, clouds, budget_bytes: int, capacity: int = 16, plans_per_cloud: int = 1,
                 tune=None, device="cuda", min_plan_views: int = 2, streams: int = 2):
        import torch
        self.torch = torch
        self.device = device
        self.min_plan_views = min_plan_views
        self.clouds = clouds
        self.capacity = capacity
        self.arena_mem = torch.empty(budget_bytes, dtype=torch.uint8, device=device)
        self.base = self.arena_mem.data_ptr()
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, streams))]
        self.stream_busy = [None] * len(self.streams)     # completion event of the batch on it
        self.plans = [[pcr.BatchPlan(c, capacity, tune=tune, stream=self.streams[0])
                       for _ in range(plans_per_cloud)] for c in clouds]
        self.plan_busy = [[False] * plans_per_cloud for _ in clouds]
        self.points = [pcr._npoints(c) for c in clouds]

    def bytes_for(self, req: Request) -> int:
        """Framebuffer bytes of a request; raises pcr.PcrError for a request
        that no batch plan can render (so that it is refused alone instead
        of failing the batch it would join)."""
        nb = pcr.fb_bytes(req.w, req.h, req.variant)
        if nb == 0:
            raise pcr.PcrError(pcr.EINVAL, pcr.lib().pcr_last_error().decode())
        if req.variant & (pcr.F_HQ_PACKED | pcr.F_HQ_ROBUST):
            raise pcr.PcrError(pcr.EUNSUPPORTED,
                               "served requests use the two-word HQ sums (no F_HQ_PACKED or F_HQ_ROBUST)")
        if req.w * req.h >= 1 << 27:
            raise pcr.PcrError(pcr.EINVAL, f"{req.w}x{req.h}: served views hold at most 2^27 - 1 pixels")
        if np.asarray(req.mvp).size != 16:
            raise pcr.PcrError(pcr.EINVAL, "mvp must hold 16 floats")
        return _align(nb)

    def new_image(self, req: Request):
        return self.torch.empty(req.w * req.h, dtype=self.torch.int32, device=self.device)

    def free_slot(self, cloud: int):
        """(plan, stream), both free, or None."""
        try:
            si = self.stream_busy.index(None)
            pi = self.plan_busy[cloud].index(False)
        except ValueError:
            return None
        return pi, si

    def launch(self, cloud: int, slot, reqs, offsets, images):
        pi, si = slot
        plan, stream = self.plans[cloud][pi], self.streams[si]
        for img in images:
            img.record_stream(stream)
        # a marker range per batch for rocprofv3's marker trace (roctx)
        self.torch.cuda.nvtx.range_push(f"serve cloud {cloud}: {len(reqs)} views, stream {si}")
        try:
            if len(reqs) < self.min_plan_views:
                # Too few views to share the point stream: the single-view
                # path (same images), enqueued without any host
                # synchronisation.
                for r, off, img in zip(reqs, offsets, images):
                    v = pcr.DEDUP if r.variant == pcr.BASIC else r.variant
                    fb = self.base + off
                    pcr.fb_clear(fb, r.w, r.h, v, stream=stream)
                    pcr.render(self.clouds[cloud], r.mvp, r.w, r.h, v, fb, stream=stream)
                    pcr.resolve(fb, r.w, r.h, v, out=img, stream=stream)
            else:
                views = [pcr.make_view(r.mvp, r.w, r.h, r.variant, self.base + off, img)
                         for r, off, img in zip(reqs, offsets, images)]
                plan.launch(views, stream=stream)
        except Exception:
            # Work enqueued before the failure may still write into these
            # framebuffers: let it finish before the caller hands their
            # memory to other requests.
            stream.synchronize()
            raise
        finally:
            self.torch.cuda.nvtx.range_pop()
        ev = self.torch.cuda.Event()
        ev.record(stream)
        self.stream_busy[si] = ev
        self.plan_busy[cloud][pi] = True
        return (cloud, pi, si)

    def done(self, handle) -> bool:
        ev = self.stream_busy[handle[2]]
        return ev is None or ev.query()

    def retire(self, handle):
        cloud, pi, si = handle
        self.stream_busy[si] = None
        self.plan_busy[cloud][pi] = False

    def close(self):
        for row in self.plans:
            for plan in row:
                plan.close()


class Server:
    """Continuous-batching scheduler (see the module docstring).

    submit() may be called from any thread; results are delivered through
    futures.  start() runs the loop in a thread of its own; without it the
    caller drives the loop with step() or drain()."""

    def __init__(self, backend, budget_bytes: int, max_batch: int | None = None, poll_s: float = 2e-5,
                 max_batch_points: int | None = None, big_points: int | None = None,
                 small_beside_big: int | None = None):
        self.be = backend
        self.arena = Arena(budget_bytes)
        self.max_batch = max_batch or backend.capacity
        # A batch completes as a whole: on a large cloud, fewer views per batch
        # keep its first request from waiting for the others' frames.
        self.max_batch_points = max_batch_points
        # Batches that stream at least big_points points (an HQ view streams
        # its cloud twice) run one at a time in arrival order, beside any
        # number of smaller batches: a large frame is not stretched by another
        # large frame, and small requests never wait for one.
        self.big_points = big_points
        # At most this many smaller batches in flight while a large one runs
        # (None: no limit): each of them takes a share of the device from it.
        self.small_beside_big = small_beside_big
        self.poll_s = poll_s
        self.lock = threading.Lock()
        self.incoming = []            # (request, future) not yet admitted, arrival order
        self.admitted = {}            # cloud -> list of (request, future, offset, image)
        self.inflight = []            # (handle, [(request, future, offset, image)], launched, big)
        self.next_id = 0
        self.completed = 0
        self.rejected = 0
        self._stop = False
        self._thread = None

    # -- client side ----------------------------------------------------------
    def submit(self, req: Request) -> Future:
        fut = Future()
        with self.lock:
            req.rid = self.next_id
            self.next_id += 1
            if req.arrival == 0.0:
                req.arrival = time.perf_counter()
            why = ""
            if not (0 <= req.cloud < len(self.be.points)):
                why = "unknown cloud"
            else:
                try:
                    if self.be.bytes_for(req) > self.arena.size:
                        why = "request does not fit the framebuffer budget"
                except Exception as e:  # a request the backend cannot render
                    why = f"invalid request: {e}"
            if why:
                self.rejected += 1
                fut.set_result(Result(req.rid, None, req.arrival, 0.0, time.perf_counter(), 0, "rejected", why))
                return fut
            self.incoming.append((req, fut))
        return fut

    # -- scheduler ------------------------------------------------------------
    def _admit(self):
        with self.lock:
            keep = []
            blocked = False
            for req, fut in self.incoming:
                if fut.cancelled():
                    continue
                off = None if blocked else self.arena.alloc(self.be.bytes_for(req))
                if off is None:
                    blocked = True     # arrival order: later requests wait behind it
                    keep.append((req, fut))
                    continue
                self.admitted.setdefault(req.cloud, []).append((req, fut, off, self.be.new_image(req)))
            self.incoming = keep

    def _batch_limit(self, cloud: int) -> int:
        if not self.max_batch_points:
            return self.max_batch
        return max(1, min(self.max_batch, self.max_batch_points // max(1, self.be.points[cloud])))

    def _streamed_points(self, cloud: int, reqs) -> int:
        return self.be.points[cloud] * sum(2 if r.variant == pcr.HQ else 1 for r in reqs)

    def _launch(self):
        big_busy = any(item[3] for item in self.inflight)
        small = len(self.inflight) - sum(1 for item in self.inflight if item[3])
        # the cloud of the oldest waiting request first
        waiting = sorted((items[0][0].rid, cloud) for cloud, items in self.admitted.items() if items)
        for _, cloud in waiting:
            items = self.admitted[cloud]
            k = self._batch_limit(cloud)
            take, rest = items[:k], items[k:]
            big = (self.big_points is not None and
                   self._streamed_points(cloud, [t[0] for t in take]) >= self.big_points)
            if big and big_busy:
                continue
            if (not big and big_busy and self.small_beside_big is not None
                    and small >= self.small_beside_big):
                continue
            slot = self.be.free_slot(cloud)
            if slot is None:
                continue
            self.admitted[cloud] = rest
            now = time.perf_counter()
            try:
                h = self.be.launch(cloud, slot, [t[0] for t in take], [t[2] for t in take],
                                   [t[3] for t in take])
            except Exception as e:  # a failed launch fails its requests; the server goes on
                for req, fut, off, _ in take:
                    self.arena.release(off, self.be.bytes_for(req))
                    fut.set_result(Result(req.rid, None, req.arrival, now, time.perf_counter(), len(take),
                                          "error", str(e)))
                continue
            self.inflight.append((h, take, now, big))
            big_busy |= big
            small += not big

    def _complete(self):
        still = []
        for item in self.inflight:
            h, take, launched, _ = item
            if not self.be.done(h):
                still.append(item)
                continue
            fin = time.perf_counter()
            self.be.retire(h)
            for req, fut, off, img in take:
                self.arena.release(off, self.be.bytes_for(req))
                self.completed += 1
                fut.set_result(Result(req.rid, img, req.arrival, launched, fin, len(take)))
        self.inflight = still

    def step(self) -> bool:
        """One scheduler iteration; True while work is pending."""
        self._complete()
        self._admit()
        self._launch()
        with self.lock:
            pending = bool(self.incoming) or any(self.admitted.values())
        return pending or bool(self.inflight)

    def drain(self, timeout_s: float = 60.0):
        t0 = time.perf_counter()
        while self.step():
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError("server did not drain")
            time.sleep(self.poll_s)

    def start(self):
        def loop():
            while not self._stop:
                busy = self.step()
                if not busy:
                    time.sleep(self.poll_s)
        self._thread = threading.Thread(target=loop, daemon=True)
        self._thread.start()

    def stop(self):
        self._stop = True
        if self._thread:
            self._thread.join()
        self.drain()


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")
