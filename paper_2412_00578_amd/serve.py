"""Continuous-batching render server over resident scenes.

Several scenes stay resident in HBM.  Render requests (scene, camera at any
resolution) arrive over time; the scheduler admits waiting requests into a
batch while the batch's estimated device footprint fits the memory pool and a
launch slot is free, and renders each batch with one launch per stage of the
batched C ABI (``ss_batch_begin`` / ``ss_batch_finish``): records of all the
batch's scenes in one preprocess, one scan, one key emission with
batch-global tile ids, one sort, one tile-range pass and one blend that
writes every request's image.  Batches alternate between launch slots (HIP
streams of default priority), so a new batch's preprocess and sort overlap the
previous batch's blend, and requests that arrive while others are on the GPU
join the next batch as soon as a slot and memory free up.

An item's pairs, sorted and blended inside a batch, are exactly the pairs it
has alone, so every served image is bit-identical to rendering the request by
itself.

The scheduler is independent of the device: ``GpuBackend`` renders on the
GPU; tests drive the same scheduler with a mock backend and a fake clock.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    scene: int
    cam: object                 # camera (width, height, fx, fy, cx, cy, R, t, near, bg)
    arrival: float              # seconds from the start of the run
    t_start: float = math.nan   # launch time of its batch
    t_done: float = math.nan    # completion time
    status: str = "pending"     # pending | done | failed
    error: str = ""
    n_pairs: int = 0
    image: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclass
class ServeStats:
    n: int
    wall_s: float
    latencies_ms: np.ndarray
    batch_sizes: list = field(default_factory=list)
    peak_reserved_bytes: int = 0
    failed: int = 0
    requeued: int = 0
    admission_bound: int = 0      # batches closed because the next request did not fit the pool
    peak_device_bytes: int = 0    # device memory the backend actually held at its peak

    def pct(self, q) -> float:
        return float(np.percentile(self.latencies_ms, q)) if len(self.latencies_ms) else math.nan

    @property
    def fps(self) -> float:
        return (self.n - self.failed) / self.wall_s if self.wall_s > 0 else math.nan

    def summary(self) -> dict:
        return {"requests": self.n, "failed": self.failed, "requeued": self.requeued,
                "wall_s": round(self.wall_s, 4), "fps": round(self.fps, 2),
                "p50_ms": round(self.pct(50), 3), "p99_ms": round(self.pct(99), 3),
                "mean_batch": round(float(np.mean(self.batch_sizes)), 2) if self.batch_sizes
                else 0.0,
                "peak_reserved_gib": round(self.peak_reserved_bytes / 2**30, 3),
                "admission_bound_batches": self.admission_bound,
                "peak_device_gib": round(self.peak_device_bytes / 2**30, 3)}


class Scheduler:
    """Admission by memory footprint, continuous batching over launch slots.

    backend must provide
      footprint(req) -> int            estimated device bytes while in flight
      launch(batch, slot) -> handle    start a batch (may raise: the batch fails;
                                       WorkspaceTooSmall re-queues its requests)
      bytes_in_flight(handle) -> int   exact device bytes of a launched batch
      done(handle) -> bool             non-blocking completion test
      wait(handle)                     block until done
      complete(handle) -> list[float]  completion time of each request (clock s)
      release(handle)                  drop the batch's buffers
    clock() -> seconds; sleep(s)."""

    def __init__(self, backend, pool_bytes: int, max_batch: int = 8, slots: int = 2,
                 clock=time.perf_counter, sleep=time.sleep, max_retries: int = 2):
        self.backend = backend
        self.pool_bytes = int(pool_bytes)
        self.max_batch = int(max_batch)
        self.slots = int(slots)
        self.clock = clock
        self.sleep = sleep
        self.max_retries = max_retries

    def run(self, requests: list[Request], skip: int = 0) -> ServeStats:
        """Serves every request; the statistics cover the requests after the
        first `skip` arrivals (a warm-up that still loads the server), with the
        rate taken from the first counted arrival to the last counted
        completion."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        now = lambda: self.clock() - t0
        pending: collections.deque = collections.deque()
        inflight = []                     # [handle, batch, reserved bytes, slot]
        free_slots = list(range(self.slots))
        reserved = peak = 0
        nxt = finished = failed = requeued = 0
        sizes = []
        bound = 0
        retries = collections.Counter()
        while finished < len(reqs):
            while nxt < len(reqs) and reqs[nxt].arrival <= now():
                pending.append(reqs[nxt])
                nxt += 1
            # retire completed batches: release their memory and slot
            keep = []
            for rec in inflight:
                h, batch, nbytes, slot = rec
                if self.backend.done(h):
                    for r, t in zip(batch, self.backend.complete(h)):
                        r.t_done = t - t0
                        r.status = "done"
                    self.backend.release(h)
                    reserved -= nbytes
                    free_slots.append(slot)
                    finished += len(batch)
                else:
                    keep.append(rec)
            inflight = keep
            # admit waiting requests, in arrival order, while they fit the pool
            launched = False
            if free_slots and pending:
                batch, nbytes = [], 0
                while pending and len(batch) < self.max_batch:
                    fb = self.backend.footprint(pending[0])
                    if reserved + nbytes + fb > self.pool_bytes:
                        if not batch and not inflight:
                            batch.append(pending.popleft())   # alone in an empty pool
                            nbytes += fb
                        else:
                            bound += 1
                        break
                    batch.append(pending.popleft())
                    nbytes += fb
                if batch:
                    slot = free_slots.pop()
                    start = now()
                    try:
                        h = self.backend.launch(batch, slot)
                    except Exception as e:  # the batch fails; the server keeps going
                        free_slots.append(slot)
                        for r in reversed(batch):
                            retries[r.rid] += 1
                            if _retryable(e) and retries[r.rid] <= self.max_retries:
                                pending.appendleft(r)
                                requeued += 1
                            else:
                                r.status, r.error, r.t_done = "failed", str(e), now()
                                failed += 1
                                finished += 1
                        continue
                    for r in batch:
                        r.t_start = start
                    # the exact size is known once the batch's pair count is
                    nbytes = max(nbytes, int(self.backend.bytes_in_flight(h)))
                    reserved += nbytes
                    peak = max(peak, reserved)
                    inflight.append([h, batch, nbytes, slot])
                    sizes.append(len(batch))
                    launched = True
            if launched:
                continue
            if inflight and (not free_slots or pending):
                self.backend.wait(inflight[0][0])       # blocked on a slot or on memory
            elif inflight:
                t_next = reqs[nxt].arrival if nxt < len(reqs) else math.inf
                self.sleep(max(0.0, min(t_next - now(), 1e-4)))
            elif nxt < len(reqs):
                self.sleep(max(0.0, reqs[nxt].arrival - now()))
        counted = reqs[skip:]
        lat = np.array([(r.t_done - r.arrival) * 1e3 for r in counted if r.status == "done"])
        wall = now()
        if skip and counted:
            wall = max(r.t_done for r in counted) - counted[0].arrival
        n_failed = sum(r.status == "failed" for r in counted)
        peak_dev = getattr(self.backend, "peak_device_bytes", lambda: 0)()
        return ServeStats(len(counted), wall, lat, sizes, peak, n_failed, requeued, bound,
                          peak_dev)


class WorkspaceTooSmall(RuntimeError):
    """Raised by a backend when a batch needs more pairs than it reserved."""


def _retryable(e) -> bool:
    return isinstance(e, WorkspaceTooSmall)


class GpuBackend:
    """Renders batches on the GPU with the batched C ABI, one HIP stream per
    launch slot; the footprint estimate uses the last pair count seen per
    (scene, resolution).  (Running each batch's depth order and scan on a
    third stream, as render_many does for frames, measured no gain here.)"""

    def __init__(self, scenes, device="cuda", mode="accutile", keep_images=False):
        import torch

        from .render import BatchRenderer
        self.torch = torch
        self.scenes = scenes
        self.device = torch.device(device)
        self.mode = mode
        self.keep_images = keep_images
        self.br = BatchRenderer(self.device)
        self.streams = {}
        self.pairs_per = {}
        self.ref_event = None
        self.ref_clock = None

    def _stream(self, slot):
        if slot not in self.streams:
            self.streams[slot] = self.torch.cuda.Stream(self.device)
        return self.streams[slot]

    def _key(self, r):
        return (r.scene, int(r.cam.width), int(r.cam.height))

    def footprint(self, r) -> int:
        n = self.scenes[r.scene].n
        px = int(r.cam.width) * int(r.cam.height)
        est = self.pairs_per.get(self._key(r), 4 * n)
        # records 48, counts 4, tile sets 16, depth keys 8, order 8, counts in
        # depth order 4, offsets 4, emit scratch 24 (tile sets in depth order,
        # the queue and its part counters): 116 B per slot; image and
        # per-pixel state 20 B per pixel (budgeted at 32 with the per-tile
        # ranges and order); 16 B per pair (two buffers) with the 1.25 growth;
        # sort scratch
        return int(116 * n + 32 * px + 16 * 1.25 * est + (3 << 20))

    def peak_device_bytes(self) -> int:
        """Device memory the batches held at the peak of the run, beyond what
        was allocated when the run started (the resident scenes)."""
        torch = self.torch
        return max(0, int(torch.cuda.max_memory_allocated(self.device)) - self.base_bytes)

    def sync_reference(self, clock):
        """Ties GPU event times to the scheduler clock."""
        torch = self.torch
        torch.cuda.synchronize(self.device)
        self.base_bytes = int(torch.cuda.memory_allocated(self.device))
        torch.cuda.reset_peak_memory_stats(self.device)
        self.ref_event = torch.cuda.Event(enable_timing=True)
        self.ref_event.record(torch.cuda.current_stream(self.device))
        torch.cuda.synchronize(self.device)
        self.ref_clock = clock()

    def launch(self, batch, slot):
        torch = self.torch
        st = self._stream(slot)
        with torch.cuda.stream(st):
            reqs = [(self.scenes[r.scene], r.cam) for r in batch]
            h = self.br.begin(reqs, self.mode, stream=st)
            per = h.n_pairs / max(len(batch), 1)
            for r in batch:
                self.pairs_per[self._key(r)] = per
                r.n_pairs = int(per)
            self.br.finish(h)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(st)
        return (h, ev, batch)

    def bytes_in_flight(self, handle) -> int:
        return handle[0].nbytes

    def done(self, handle) -> bool:
        return handle[1].query()

    def wait(self, handle):
        handle[1].synchronize()

    def complete(self, handle):
        h, ev, batch = handle
        t = self.ref_clock + self.ref_event.elapsed_time(ev) * 1e-3
        if self.keep_images:
            for r, img in zip(batch, h.outs):
                r.image = img
        return [t] * len(batch)

    def release(self, handle):
        pass


def serve(scenes, requests, device="cuda", mode="accutile", pool_bytes=16 << 30, max_batch=8,
          slots=2, keep_images=False, skip=0) -> ServeStats:
    """Runs the request stream against resident scenes in real time; the
    statistics leave out the first `skip` arrivals."""
    backend = GpuBackend(scenes, device, mode, keep_images)
    sched = Scheduler(backend, pool_bytes, max_batch, slots)
    backend.sync_reference(sched.clock)
    return sched.run(requests, skip)
