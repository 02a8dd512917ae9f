"""Continuous-batching view server over resident scenes.

Scenes stay resident in device memory.  Requests (scene, camera) arrive over
time; the scheduler admits the oldest pending requests into a batch while a
stream slot is free and the batch's exact workspace bytes fit the HBM budget,
renders the batch as ONE multi-view plan (mixed resolutions and scenes in the
same launches) on that stream, and moves on: requests that arrive while
earlier batches run form the next batch, whose projection/sort/binning
overlaps the previous batch's compositing on another stream.  Completion is
stamped from a HIP event on the GPU clock, so a request's latency is
(completion - arrival) without host polling delay.

Every view's result is independent of its batch-mates (its items, depth
order, tile lists and arithmetic do not depend on them), so a request renders
bit-identically alone and in any mix.

The scheduler is plain Python over an executor interface; `RendererExecutor`
drives libdpr through the binding, `SimulatedExecutor` stands in for it in CPU
tests of the scheduling logic.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    scene: int
    camera: object            # R, t, fx, fy, cx, cy, width, height
    arrival: float            # seconds on the server clock
    done: Optional[float] = None
    batch: int = -1
    image: object = None      # device tensor [H, W, 3] once rendered
    trans: object = None
    error: Optional[str] = None

    @property
    def pixels(self) -> int:
        return int(self.camera.width) * int(self.camera.height)

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


@dataclasses.dataclass
class Batch:
    bid: int
    requests: List[Request]
    slot: int
    nbytes: int
    handle: object = None


class SimulatedExecutor:
    """Executor with a linear cost model (for CPU tests of the scheduler):
    a batch takes `fixed + per_pixel * pixels` seconds after it is launched on
    a free slot; workspace bytes are `bytes_per_pixel * pixels`."""

    def __init__(self, n_slots=2, fixed=0.002, per_pixel=1e-9, bytes_per_pixel=16, fail_scene=None):
        self.n_slots = n_slots
        self.fixed, self.per_pixel, self.bpp = fixed, per_pixel, bytes_per_pixel
        self.fail_scene = fail_scene
        self.clock: Callable[[], float] = time.perf_counter
        self.launched = []

    def request_bytes(self, req: Request) -> int:
        return self.bpp * req.pixels

    def start(self, batch: Batch, now: float):
        if self.fail_scene is not None and any(r.scene == self.fail_scene for r in batch.requests):
            raise RuntimeError("simulated launch failure")
        px = sum(r.pixels for r in batch.requests)
        self.launched.append((now, [r.rid for r in batch.requests]))
        return now + self.fixed + self.per_pixel * px

    def poll(self, batch: Batch, now: float) -> Optional[float]:
        return batch.handle if now >= batch.handle else None

    def finish(self, batch: Batch):
        pass


class RendererExecutor:
    """Runs batches with libdpr: one multi-view plan per batch, on one of
    `n_slots` HIP streams (default priority)."""

    def __init__(self, scenes, params=None, n_slots=2, device="cuda"):
        import torch
        from .renderer import Plan, RenderParams
        self.torch = torch
        self.Plan = Plan
        self.scenes = list(scenes)
        self.params = params or RenderParams(bwd_mode="recompute")
        self.n_slots = n_slots
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_slots)]
        self.device = device
        self.lib = None
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record()
        self.ref.synchronize()
        self.ref_host = time.perf_counter()
        self.clock: Callable[[], float] = time.perf_counter

    def _ws_bytes(self, scene_ids, cams):
        from . import _abi
        from .renderer import camera_struct
        L = _abi.load()
        c_scenes = (_abi.Scene * len(self.scenes))(*[s.c_struct() for s in self.scenes])
        views = (_abi.View * len(cams))(*[_abi.View(int(si), 0, camera_struct(c), 1, 0)
                                        for si, c in zip(scene_ids, cams)])
        return int(L.dpr_plan_ws_bytes(c_scenes, len(self.scenes), views, len(cams)))

    def request_bytes(self, req: Request) -> int:
        # exact plan workspace + image + a pair-list bound (4 B per pair, with the
        # scene's points covering at most 64 tiles each)
        plan = self._ws_bytes([req.scene], [req.camera])
        n = self.scenes[req.scene].n
        return plan + 12 * req.pixels + 4 * n * 64 + 8 * req.pixels

    def start(self, batch: Batch, now: float):
        torch = self.torch
        st = self.streams[batch.slot]
        with torch.cuda.stream(st):
            plan = self.Plan(self.scenes, [(r.scene, r.camera) for r in batch.requests], self.params, stream=st,
                             trans=[None] * len(batch.requests))
            plan.forward()
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(st)
        for r, img in zip(batch.requests, plan.images):
            r.image = img
        return (plan, ev)

    def exact_bytes(self, batch: Batch) -> int:
        """Device bytes the batch really holds (known once its plan stage ran)."""
        plan, _ = batch.handle
        inf = plan.info()
        return int(inf.plan_ws_bytes + inf.fwd_ws_bytes) + sum(12 * r.pixels for r in batch.requests)

    def poll(self, batch: Batch, now: float) -> Optional[float]:
        plan, ev = batch.handle
        if not ev.query():
            return None
        return self.ref_host + self.ref.elapsed_time(ev) / 1e3

    def finish(self, batch: Batch):
        plan, _ = batch.handle
        plan.free()


class Server:
    """Continuous batching: FIFO admission under a slot limit, a view limit per
    batch and an HBM budget (bytes)."""

    def __init__(self, executor, hbm_budget: int, max_views: int = 32):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_views = max_views
        self.pending: Deque[Request] = collections.deque()
        self.inflight: List[Batch] = []
        self.finished: List[Request] = []
        self.in_use = 0
        self.peak_in_use = 0
        self.next_bid = 0
        self.batches: List[int] = []

    def submit(self, req: Request):
        self.pending.append(req)

    def _free_slot(self) -> Optional[int]:
        busy = {b.slot for b in self.inflight}
        for s in range(self.ex.n_slots):
            if s not in busy:
                return s
        return None

    def _admit(self, now: float) -> bool:
        slot = self._free_slot()
        if slot is None or not self.pending:
            return False
        reqs, nbytes = [], 0
        while self.pending and len(reqs) < self.max_views:
            r = self.pending[0]
            b = self.ex.request_bytes(r)
            if self.in_use + nbytes + b > self.budget and (reqs or self.inflight):
                break                       # wait for memory to free up
            reqs.append(self.pending.popleft())
            nbytes += b
        if not reqs:
            return False
        batch = Batch(self.next_bid, reqs, slot, nbytes)
        self.next_bid += 1
        try:
            batch.handle = self.ex.start(batch, now)
        except Exception as e:              # failed launch: the requests fail, nothing is held
            for r in reqs:
                r.error = str(e)
                r.done = now
                self.finished.append(r)
            return True
        for r in reqs:
            r.batch = batch.bid
        exact = getattr(self.ex, "exact_bytes", None)
        if exact is not None:
            batch.nbytes = exact(batch)
            nbytes = batch.nbytes
        self.inflight.append(batch)
        self.in_use += nbytes
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.batches.append(len(reqs))
        return True

    def _reap(self, now: float):
        still = []
        for b in self.inflight:
            t = self.ex.poll(b, now)
            if t is None:
                still.append(b)
                continue
            for r in b.requests:
                r.done = t
                self.finished.append(r)
            self.in_use -= b.nbytes
            self.ex.finish(b)
        self.inflight = still

    def step(self, now: float):
        self._reap(now)
        while self._admit(now):
            pass

    def idle(self) -> bool:
        return not self.pending and not self.inflight

    def run_trace(self, trace: Sequence, make_request: Callable, clock=None, spin: float = 0.0):
        """Replays `trace` (objects with .arrival seconds) in real time on
        `clock`; returns the finished requests."""
        clock = clock or self.ex.clock
        t0 = clock()
        i = 0
        n = len(trace)
        while i < n or not self.idle():
            now = clock() - t0
            while i < n and trace[i].arrival <= now:
                req = make_request(i, trace[i])
                req.arrival = t0 + trace[i].arrival
                self.submit(req)
                i += 1
            self.step(clock())
            if spin:
                time.sleep(spin)
        return self.finished


def latency_stats(reqs: Sequence[Request], wall: float) -> dict:
    ok = [r for r in reqs if r.error is None and r.latency is not None]
    lat = np.array([r.latency for r in ok]) * 1e3 if ok else np.zeros(1)
    px = sum(r.pixels for r in ok)
    return {"requests": len(reqs), "failed": len(reqs) - len(ok),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "mean_ms": float(lat.mean()),
            "served_mpix_s": px / wall / 1e6 if wall > 0 else 0.0}
