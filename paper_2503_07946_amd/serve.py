"""Continuous-batching render server for resident 7DGS scenes.

Requests (scene, camera, t) arrive over time.  The scheduler keeps a FIFO of
arrived requests and up to `max_inflight` batches on the device at once
(each on its own HIP stream, so their work overlaps).  Whenever a batch
completes or a request arrives, it forms the next batch from the head of the
queue: up to `max_slots` frames whose device-memory footprint (workspace,
pair arena, outputs) fits in what the HBM budget has free.  A frame whose
pairs overflowed the arena estimate is requeued at the head with the exact
count it reported; a request larger than the whole budget is rejected; a
request still queued at its deadline is cancelled.

The scheduler talks to an executor through five calls (estimate, launch,
ready, collect, wait); GpuExecutor runs batches through lib7dgs, and any
object with the same calls can stand in for it (the tests use a CPU fake).
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

PAIR_ROUND = 2048  # the library's SD7_PAIR_ROUND: a frame's arena share is a multiple of it


@dataclass(eq=False)       # a request is itself: compared by identity
class Request:
    rid: int
    arrival: float          # seconds since the stream started
    scene: int
    view: object
    deadline: float | None = None
    # filled in by the scheduler
    status: str = "pending"  # pending, queued, inflight, done, rejected, cancelled
    admit: float | None = None
    done: float | None = None
    attempts: int = 0
    pairs_hint: int | None = None
    result: object = None

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


@dataclass(eq=False)
class Outcome:
    req: Request
    ok: bool                 # False: pair overflow, needs a retry
    pairs: int               # pairs the frame needed
    result: object = None


@dataclass
class ServeStats:
    completed: list
    rejected: list
    cancelled: list
    batches: int
    retries: int
    wall: float
    batch_sizes: list = field(default_factory=list)

    def latencies(self, skip: int = 0):
        done = sorted(self.completed, key=lambda r: r.rid)
        return np.array([r.latency for r in done if r.rid >= skip])

    def summary(self, skip: int = 0) -> dict:
        lat = self.latencies(skip) * 1e3
        done = [r for r in self.completed if r.rid >= skip]
        span = (max(r.done for r in done) - min(r.arrival for r in done)) if done else 0.0
        return {"requests": len(done), "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_ms": float(lat.mean()) if len(lat) else None,
                "throughput_fps": len(done) / span if span > 0 else None,
                "rejected": len(self.rejected), "cancelled": len(self.cancelled),
                "batches": self.batches, "retries": self.retries,
                "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0}


class Scheduler:
    def __init__(self, executor, hbm_budget: int, max_slots: int = 16, max_inflight: int = 2,
                 clock=time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.max_inflight = int(max_inflight)
        self.clock = clock

    def run(self, requests, realtime: bool = True) -> ServeStats:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        inflight = []           # (handle, reqs, bytes)
        used = 0
        completed, rejected, cancelled = [], [], []
        batches = retries = 0
        sizes = []
        t0 = self.clock()

        def now():
            return self.clock() - t0

        while pending or queue or inflight:
            t = now()
            while pending and (pending[0].arrival <= t or not realtime):
                r = pending.popleft()
                r.status = "queued"
                queue.append(r)
            # deadlines of queued requests
            if any(r.deadline is not None and r.deadline <= t for r in queue):
                keep = collections.deque()
                for r in queue:
                    if r.deadline is not None and r.deadline <= t:
                        r.status = "cancelled"
                        cancelled.append(r)
                    else:
                        keep.append(r)
                queue = keep
            # completions
            progressed = False
            for item in list(inflight):
                h, reqs, nbytes = item
                if not self.ex.ready(h):
                    continue
                inflight = [x for x in inflight if x is not item]
                used -= nbytes
                progressed = True
                tdone = now()
                redo = []
                for o in self.ex.collect(h):
                    if o.ok:
                        o.req.status = "done"
                        o.req.done = tdone
                        o.req.result = o.result
                        completed.append(o.req)
                    else:
                        o.req.pairs_hint = o.pairs
                        o.req.status = "queued"
                        redo.append(o.req)
                        retries += 1
                for r in reversed(redo):
                    queue.appendleft(r)
            # admission: next batch from the head of the queue
            while queue and len(inflight) < self.max_inflight:
                batch, need = [], 0
                while queue and len(batch) < self.max_slots:
                    r = queue[0]
                    est = self.ex.footprint(r)
                    if est > self.budget:
                        queue.popleft()
                        r.status = "rejected"
                        rejected.append(r)
                        continue
                    if used + need + est > self.budget:
                        break
                    queue.popleft()
                    batch.append(r)
                    need += est
                if not batch:
                    break
                tl = now()
                for r in batch:
                    r.status = "inflight"
                    r.admit = tl
                    r.attempts += 1
                h, nbytes = self.ex.launch(batch)
                used += nbytes
                inflight.append((h, batch, nbytes))
                batches += 1
                sizes.append(len(batch))
                progressed = True
            if progressed:
                continue
            # idle: wait for a completion or the next arrival
            wait = None
            if pending and realtime:
                wait = max(0.0, pending[0].arrival - now())
            if inflight:
                self.ex.wait([h for h, _, _ in inflight], wait)
            elif wait is not None:
                time.sleep(min(wait, 0.05))
            elif queue:
                # nothing in flight and the head does not fit: cannot happen
                # unless the budget shrank; reject the head to make progress
                r = queue.popleft()
                r.status = "rejected"
                rejected.append(r)
        return ServeStats(completed, rejected, cancelled, batches, retries, now(), sizes)


def run_plain(executor, requests, realtime: bool = True, clock=time.perf_counter) -> ServeStats:
    """Baseline: one request at a time in arrival order, each rendered by one
    call and waited for before the next starts, on the same kernels."""
    t0 = clock()
    done = []
    for r in sorted(requests, key=lambda q: q.arrival):
        if realtime:
            while clock() - t0 < r.arrival:
                time.sleep(min(0.001, max(0.0, r.arrival - (clock() - t0))))
        r.admit = clock() - t0
        r.result = executor.render_one(r)
        r.done = clock() - t0
        r.status = "done"
        done.append(r)
    return ServeStats(done, [], [], len(done), 0, clock() - t0, [1] * len(done))


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------

class GpuExecutor:
    """Runs batches through lib7dgs on a small pool of HIP streams (default
    priority).  Footprints come from sd7_plan with a per-(scene, resolution)
    pair estimate learned from completed frames."""

    def __init__(self, renderer, scenes, nstreams: int = 2, keep_images: bool = False,
                 pair_margin: float = 1.15):
        import torch
        self.torch = torch
        self.R = renderer
        self.scenes = scenes
        self.streams = [torch.cuda.Stream(device=renderer.device) for _ in range(nstreams)]
        self.next_stream = 0
        self.keep = keep_images
        self.margin = pair_margin
        self.est = {}           # (scene, W, H) -> pairs

    # -- estimates ------------------------------------------------------------
    def pair_estimate(self, r: Request) -> int:
        if r.pairs_hint is not None:
            return int(r.pairs_hint)
        key = (r.scene, r.view.W, r.view.H)
        if key in self.est:
            return int(self.est[key] * self.margin)
        n = self.scenes[r.scene].n
        return int(100 * n * r.view.W * r.view.H / 1e6) + PAIR_ROUND

    def footprint(self, r: Request) -> int:
        pairs = (self.pair_estimate(r) + PAIR_ROUND - 1) // PAIR_ROUND * PAIR_ROUND
        n = self.scenes[r.scene].n
        px = r.view.W * r.view.H
        # workspace: per-Gaussian arrays (~200 B), pairs in two buffers plus
        # sort histograms (~17 B/pair), tile ranges; outputs 20 B/pixel
        return 200 * n + 17 * pairs + 8 * (px // 256 + 64) + 20 * px + (1 << 16)

    # -- execution -----------------------------------------------------------
    def launch(self, reqs):
        torch = self.torch
        s = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        cap = 0
        for r in reqs:
            cap += (self.pair_estimate(r) + PAIR_ROUND - 1) // PAIR_ROUND * PAIR_ROUND
        with torch.cuda.stream(s):
            frames = self.R.make_frames([(self.scenes[r.scene], r.view) for r in reqs])
            b = self.R.batch(frames, cap)
            self.R.stage("sd7_render", b, stream=s)
            counts = b.counts()
            host = torch.empty(counts.shape, dtype=counts.dtype, pin_memory=True)
            host.copy_(counts, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        nbytes = int(b.ws.numel()) + sum(20 * r.view.W * r.view.H for r in reqs)
        return (b, host, ev, list(reqs)), nbytes

    def ready(self, h) -> bool:
        return h[2].query()

    def wait(self, handles, timeout):
        # block on the oldest batch; the scheduler polls the rest
        if timeout is None or timeout > 0.002:
            handles[0][2].synchronize()

    def collect(self, h):
        from . import _lib as L
        b, host, ev, reqs = h
        c = host.numpy()
        out = []
        for k, r in enumerate(reqs):
            flags = int(c[k, L.SD7_CNT_FLAGS])
            need = int(c[k, L.SD7_CNT_NEEDED])
            ok = not (flags & L.SD7_FLAG_PAIR_OVERFLOW)
            key = (r.scene, r.view.W, r.view.H)
            self.est[key] = max(self.est.get(key, 0), need)
            res = None
            if ok and self.keep:
                fr = b.frames[k]
                res = (fr.image.cpu(), fr.final_T.cpu(), fr.last.cpu())
            out.append(Outcome(r, ok, need, res))
        return out

    def render_one(self, r: Request):
        """Plain path: one frame in one sd7_render call with the pair count
        learned for its (scene, resolution), then one wait for its counters;
        if the arena overflowed it is rendered again with the exact count."""
        from . import _lib as L
        frames = self.R.make_frames([(self.scenes[r.scene], r.view)])
        key = (r.scene, r.view.W, r.view.H)
        cap = (self.pair_estimate(r) + PAIR_ROUND - 1) // PAIR_ROUND * PAIR_ROUND
        b = self.R.batch(frames, cap)
        self.R.stage("sd7_render", b)
        c = self.R.read_counts(b)
        need = int(c[0, L.SD7_CNT_NEEDED])
        self.est[key] = max(self.est.get(key, 0), need)
        if c[0, L.SD7_CNT_FLAGS] & L.SD7_FLAG_PAIR_OVERFLOW:
            b = self.R.render_frames(frames, capacity=need, exact=True)
            self.torch.cuda.current_stream().synchronize()
        if self.keep:
            fr = b.frames[0]
            return (fr.image.cpu(), fr.final_T.cpu(), fr.last.cpu())
        return None


def budget_from_gb(gb: float) -> int:
    return int(gb * (1 << 30))


def default_requests(nreq: int, qps: float, scenes_n, seed: int = 300, resolutions=None):
    import scenegen
    res = resolutions or scenegen.SERVE_RES
    stream = scenegen.request_stream(nreq, qps, nscenes=len(scenes_n), seed=seed, resolutions=res)
    return [Request(i, q.arrival, q.scene, q.view) for i, q in enumerate(stream)]


def ceil_to(x, m):
    return int(math.ceil(x / m) * m)
