"""Continuous-batching server for many simulated laparoscope streams.

Frames arrive from several camera streams of mixed resolution (each stream is
a Poisson process).  Every shape class (frame size, Haar levels, posterior
grid) gets one or more *lanes*: a plan with its tables and scratch, a device
input slab for up to `max_batch` frames, device output maps, a HIP stream and
one captured HIP graph per batch size.  Lanes are created up front inside an
HBM budget (a class whose first lane does not fit is refused).  At run time a
frame is admitted into a lane as soon as one of its class is free: every
frame that arrived while the lane was busy goes into the next batch
(continuous batching), and lanes of different classes run concurrently on
their own streams.  Latency is completion minus arrival; completion is read
from a HIP event on the lane's stream.

The scheduling logic is independent of the device: `GpuExecutor` runs the HIP
path through the C ABI, `FakeExecutor` simulates service times on the CPU for
tests of admission, batching, ordering and failure handling.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class ShapeClass:
    height: int
    width: int
    levels: int
    grid: int
    dtype: str = "f16"

    @property
    def pixels(self) -> int:
        return self.height * self.width

    def pairs(self) -> int:
        """Algorithmic posterior pairs per frame (LL pixels x grid nodes)."""
        return (self.height >> self.levels) * (self.width >> self.levels) * self.grid * self.grid

    def frame_bytes(self) -> int:
        return self.pixels * 3 * (4 if self.dtype == "f32" else 2)


@dataclasses.dataclass
class FrameRequest:
    stream: int
    index: int
    cls: ShapeClass
    arrival: float            # seconds on the server clock
    source: int = 0           # which pre-rendered frame of the class it carries
    admitted: float = math.nan
    done: float = math.nan
    lane: int = -1
    batch: int = 0
    failed: bool = False
    waited: bool = False      # arrived while every lane of its class was busy


@dataclasses.dataclass
class Lane:
    id: int
    cls: ShapeClass
    max_batch: int
    bytes: int
    handle: object = None     # executor state
    busy: bool = False
    inflight: List[FrameRequest] = dataclasses.field(default_factory=list)
    submitted_at: float = math.nan
    busy_time: float = 0.0


class Executor:
    """Device side of the server."""

    def lane_bytes(self, cls: ShapeClass, max_batch: int) -> int:
        raise NotImplementedError

    def create_lane(self, lane: Lane) -> None:
        raise NotImplementedError

    def submit(self, lane: Lane, reqs: Sequence[FrameRequest]) -> None:
        raise NotImplementedError

    def done(self, lane: Lane) -> bool:
        raise NotImplementedError

    def completion_time(self, lane: Lane) -> float:
        """Server-clock time at which the lane's last batch finished."""
        raise NotImplementedError

    def clock(self) -> float:
        return time.perf_counter()

    def release(self, lane: Lane) -> None:
        pass


@dataclasses.dataclass
class Report:
    latencies_ms: np.ndarray
    per_class: Dict[str, Dict[str, float]]
    frames: int
    failed: int
    waited: int
    window_s: float
    pixels: int
    pairs: int
    lanes: Dict[str, int]
    refused: List[str]
    hbm_bytes: int
    hbm_budget: int
    max_queue: int
    mean_batch: float
    busy_fraction: float

    def summary(self) -> Dict[str, object]:
        lat = self.latencies_ms
        q = (lambda p: float(np.percentile(lat, p)) if lat.size else math.nan)
        return {
            "frames": self.frames, "failed": self.failed, "deferred": self.waited,
            "p50_ms": round(q(50), 3), "p99_ms": round(q(99), 3), "max_ms": round(float(lat.max()) if lat.size else math.nan, 3),
            "frames_per_s": round(self.frames / self.window_s, 2),
            "mpixel_per_s": round(self.pixels / self.window_s / 1e6, 2),
            "pairs_per_s": self.pairs / self.window_s,
            "lanes": self.lanes, "refused": self.refused,
            "hbm_bytes": self.hbm_bytes, "hbm_budget": self.hbm_budget,
            "max_queue": self.max_queue, "mean_batch": round(self.mean_batch, 3),
            "lane_busy_fraction": round(self.busy_fraction, 3),
            "per_class": self.per_class,
        }


def class_name(c: ShapeClass) -> str:
    return f"{c.width}x{c.height}/L{c.levels}/G{c.grid}/{c.dtype}"


class Server:
    """Admission, continuous batching and completion tracking."""

    def __init__(self, executor: Executor, classes: Dict[ShapeClass, int], hbm_budget: int,
                 offered: Optional[Dict[ShapeClass, float]] = None, max_lanes: int = 4):
        """classes: shape class -> max batch; offered: relative load per class
        (lanes beyond the first go to the most loaded classes first)."""
        self.ex = executor
        self.budget = int(hbm_budget)
        self.lanes: List[Lane] = []
        self.by_class: Dict[ShapeClass, List[Lane]] = {}
        self.refused: List[ShapeClass] = []
        used = 0
        offered = offered or {c: 1.0 for c in classes}
        order = sorted(classes, key=lambda c: -offered.get(c, 0.0))
        # first lane per class, most loaded first
        for c in order:
            b = self.ex.lane_bytes(c, classes[c])
            if used + b > self.budget:
                self.refused.append(c)
                continue
            self._add_lane(c, classes[c], b)
            used += b
        # extra lanes round-robin while the budget allows
        grown = True
        while grown:
            grown = False
            for c in order:
                if c in self.refused or len(self.by_class[c]) >= max_lanes:
                    continue
                b = self.ex.lane_bytes(c, classes[c])
                if used + b <= self.budget:
                    self._add_lane(c, classes[c], b)
                    used += b
                    grown = True
        self.used = used

    def _add_lane(self, c: ShapeClass, max_batch: int, nbytes: int) -> None:
        lane = Lane(len(self.lanes), c, max_batch, nbytes)
        self.ex.create_lane(lane)
        self.lanes.append(lane)
        self.by_class.setdefault(c, []).append(lane)

    def close(self) -> None:
        for lane in self.lanes:
            self.ex.release(lane)

    def _finish(self, lane: Lane, now_done: float, reqs_done: List[FrameRequest], failed: bool = False) -> None:
        for r in lane.inflight:
            r.done = now_done
            r.failed = failed
            reqs_done.append(r)
        lane.busy_time += max(0.0, now_done - lane.submitted_at)
        lane.inflight = []
        lane.busy = False

    def run(self, requests: Sequence[FrameRequest], warmup_s: float = 0.0,
            on_complete: Optional[Callable[[Lane, List[FrameRequest]], None]] = None,
            idle_sleep_s: float = 50e-6) -> Report:
        """Serve `requests` (arrival times relative to the start of the run)."""
        pending = sorted(requests, key=lambda r: r.arrival)
        queues: Dict[ShapeClass, Deque[FrameRequest]] = {c: deque() for c in self.by_class}
        done: List[FrameRequest] = []
        refused = set(self.refused)
        i = 0
        t0 = self.ex.clock()
        max_queue = 0
        batches = []
        while i < len(pending) or any(queues[c] for c in queues) or any(l.busy for l in self.lanes):
            now = self.ex.clock() - t0
            # arrivals
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                i += 1
                if r.cls in refused or r.cls not in queues:
                    r.failed = True
                    done.append(r)
                    continue
                if not any(not l.busy for l in self.by_class[r.cls]) or queues[r.cls]:
                    r.waited = True
                queues[r.cls].append(r)
            # completions
            for lane in self.lanes:
                if lane.busy and self.ex.done(lane):
                    finished = list(lane.inflight)
                    self._finish(lane, self.ex.completion_time(lane) - t0, done)
                    if on_complete is not None:
                        on_complete(lane, finished)
            # admissions: every free lane takes the oldest queued frames of its class
            progressed = False
            for c, q in queues.items():
                max_queue = max(max_queue, len(q))
                for lane in self.by_class[c]:
                    if not q:
                        break
                    if lane.busy:
                        continue
                    batch = [q.popleft() for _ in range(min(lane.max_batch, len(q)))]
                    now = self.ex.clock() - t0
                    for r in batch:
                        r.admitted = now
                        r.lane = lane.id
                        r.batch = len(batch)
                    lane.inflight = batch
                    lane.busy = True
                    lane.submitted_at = now
                    batches.append(len(batch))
                    try:
                        self.ex.submit(lane, batch)
                    except Exception:
                        # a failed submission fails only its own frames; the lane is reused
                        self._finish(lane, self.ex.clock() - t0, done, failed=True)
                    progressed = True
            if not progressed:
                nxt = pending[i].arrival - (self.ex.clock() - t0) if i < len(pending) else idle_sleep_s
                if nxt > 0:
                    time.sleep(min(nxt, idle_sleep_s))
        end = max([r.done for r in done if not math.isnan(r.done)] + [0.0])
        measured = [r for r in done if r.arrival >= warmup_s and not r.failed]
        lat = np.array([(r.done - r.arrival) * 1e3 for r in measured])
        window = max(1e-9, end - warmup_s)
        per_class: Dict[str, Dict[str, float]] = {}
        for c in self.by_class:
            lc = np.array([(r.done - r.arrival) * 1e3 for r in measured if r.cls == c])
            per_class[class_name(c)] = {
                "frames": int(lc.size),
                "p50_ms": round(float(np.percentile(lc, 50)), 3) if lc.size else math.nan,
                "p99_ms": round(float(np.percentile(lc, 99)), 3) if lc.size else math.nan,
                "lanes": len(self.by_class[c]),
            }
        busy = sum(l.busy_time for l in self.lanes) / max(1e-9, end) / max(1, len(self.lanes))
        return Report(
            latencies_ms=lat, per_class=per_class, frames=len(measured),
            failed=sum(1 for r in done if r.failed), waited=sum(1 for r in measured if r.waited),
            window_s=window, pixels=sum(r.cls.pixels for r in measured),
            pairs=sum(r.cls.pairs() for r in measured),
            lanes={class_name(c): len(v) for c, v in self.by_class.items()},
            refused=[class_name(c) for c in self.refused], hbm_bytes=self.used, hbm_budget=self.budget,
            max_queue=max_queue, mean_batch=float(np.mean(batches)) if batches else 0.0,
            busy_fraction=busy)


# -----------------------------------------------------------------------------
# Executors
# -----------------------------------------------------------------------------

class FakeExecutor(Executor):
    """CPU stand-in: a batch of b frames of class c takes cost(c, b) seconds on
    its lane; `fail` decides whether a submission raises."""

    def __init__(self, cost: Callable[[ShapeClass, int], float],
                 lane_bytes: Callable[[ShapeClass, int], int] = lambda c, b: c.frame_bytes() * b * 4,
                 fail: Optional[Callable[[Lane, Sequence[FrameRequest]], bool]] = None):
        self.cost = cost
        self._bytes = lane_bytes
        self.fail = fail
        self.submissions: List[Tuple[int, List[Tuple[int, int]]]] = []

    def lane_bytes(self, cls, max_batch):
        return self._bytes(cls, max_batch)

    def create_lane(self, lane):
        lane.handle = {"done_at": 0.0}

    def submit(self, lane, reqs):
        if self.fail is not None and self.fail(lane, reqs):
            raise RuntimeError("injected failure")
        self.submissions.append((lane.id, [(r.stream, r.index) for r in reqs]))
        lane.handle["done_at"] = self.clock() + self.cost(lane.cls, len(reqs))

    def done(self, lane):
        return self.clock() >= lane.handle["done_at"]

    def completion_time(self, lane):
        return lane.handle["done_at"]


class GpuExecutor(Executor):
    """Runs batches through the C ABI on cuda:0.  `sources[c]` holds the
    pre-rendered frames of class c in pinned host memory ([n][H][W][3]; int16
    bit patterns for bfloat16)."""

    def __init__(self, spectra, sources, sigma: float = 0.01, lam: float = 1e-3, keep_outputs=None):
        import torch
        from paper_1706_07263_amd import hb
        self.torch = torch
        self.hb = hb
        self.spectra = spectra
        self.sources = sources
        self.sigma = sigma
        self.lam = lam
        self.keep = keep_outputs   # callable(req) -> bool: copy that frame's maps to host
        self.kept: Dict[Tuple[int, int], np.ndarray] = {}
        self.dev = torch.device("cuda:0")
        # reference event: server-clock time of a GPU timestamp
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        self.ref_host = time.perf_counter()

    def _torch_dtype(self, c):
        t = self.torch
        return {"f32": t.float32, "f16": t.float16, "bf16": t.int16}[c.dtype]

    def _desc(self, c: ShapeClass, max_batch: int):
        return self.hb.make_desc(c.width, c.height, levels=c.levels, dtype=c.dtype, max_batch=max_batch,
                                 grid_thb=c.grid, grid_so2=c.grid, lam=self.lam, sigma=self.sigma)

    def lane_bytes(self, cls, max_batch):
        # plan tables + scratch (asked from a throw-away plan) + input slab + 4 map slabs
        with self.hb.Plan(self._desc(cls, max_batch), 0) as p:
            plan_bytes = p.device_bytes()
        return plan_bytes + max_batch * (cls.frame_bytes() + 16 * cls.pixels)

    def create_lane(self, lane):
        t = self.torch
        c = lane.cls
        B = lane.max_batch
        plan = self.hb.Plan(self._desc(c, B), 0).set_forward_model(self.spectra)
        stream = t.cuda.Stream(self.dev)
        inp = t.zeros((B, c.height, c.width, 3), dtype=self._torch_dtype(c), device=self.dev)
        maps = [t.zeros((B, c.height, c.width), dtype=t.float32, device=self.dev) for _ in range(4)]
        graphs = {}
        with t.cuda.stream(stream):
            for b in range(1, B + 1):
                plan.estimate(inp[:b], [m[:b] for m in maps], stream)     # eager warm-up
        stream.synchronize()
        for b in range(1, B + 1):
            g = t.cuda.CUDAGraph()
            with t.cuda.graph(g, stream=stream):
                plan.estimate(inp[:b], [m[:b] for m in maps], stream)
            graphs[b] = g
        stream.synchronize()
        lane.handle = {"plan": plan, "stream": stream, "inp": inp, "maps": maps, "graphs": graphs,
                       "done": t.cuda.Event(enable_timing=True), "copies": []}

    def submit(self, lane, reqs):
        t = self.torch
        h = lane.handle
        b = len(reqs)
        with t.cuda.stream(h["stream"]):
            for i, r in enumerate(reqs):
                h["inp"][i].copy_(self.sources[r.cls][r.source], non_blocking=True)
            h["graphs"][b].replay()
            h["copies"] = []
            if self.keep is not None:
                for i, r in enumerate(reqs):
                    if self.keep(r):
                        out = t.empty((4, r.cls.height, r.cls.width), dtype=t.float32, pin_memory=True)
                        for k in range(4):
                            out[k].copy_(h["maps"][k][i], non_blocking=True)
                        h["copies"].append(((r.stream, r.index), out))
            h["done"].record(h["stream"])

    def done(self, lane):
        ok = lane.handle["done"].query()
        if ok:
            for key, out in lane.handle["copies"]:
                self.kept[key] = out.numpy().copy()
            lane.handle["copies"] = []
        return ok

    def completion_time(self, lane):
        return self.ref_host + self.ref.elapsed_time(lane.handle["done"]) / 1e3

    def release(self, lane):
        if lane.handle is not None:
            lane.handle["stream"].synchronize()
            lane.handle["plan"].close()
            lane.handle = None

    def run_alone(self, cls: ShapeClass, source: int, max_batch: int) -> np.ndarray:
        """The same frame through a fresh plan of the same class, alone (eager)."""
        t = self.torch
        with self.hb.Plan(self._desc(cls, max_batch), 0) as plan:
            plan.set_forward_model(self.spectra)
            inp = self.sources[cls][source].to(self.dev)[None]
            maps = [t.zeros((1, cls.height, cls.width), dtype=t.float32, device=self.dev) for _ in range(4)]
            plan.estimate(inp, maps)
            t.cuda.synchronize()
            return np.stack([m[0].cpu().numpy() for m in maps])


# -----------------------------------------------------------------------------
# The 16-stream workload
# -----------------------------------------------------------------------------

def workload_requests(duration_s: float, classes: Sequence[Tuple[int, int, int, int, int]] = None,
                      fps: float = 30.0, dtype: str = "f16", n_sources: int = 1
                      ) -> Tuple[List[FrameRequest], Dict[ShapeClass, float]]:
    """Poisson arrivals for the mixed-resolution streams; returns the requests
    and the offered pairs/s per class."""
    from paper_1706_07263_amd import synth
    classes = classes or synth.SERVE_CLASSES
    reqs: List[FrameRequest] = []
    offered: Dict[ShapeClass, float] = {}
    s = 0
    for count, h, w, lv, g in classes:
        c = ShapeClass(h, w, lv, g, dtype)
        for _ in range(count):
            t = synth.poisson_arrivals(s, fps, duration_s)
            for k, a in enumerate(t):
                reqs.append(FrameRequest(stream=s, index=k, cls=c, arrival=float(a), source=(s + k) % n_sources))
            offered[c] = offered.get(c, 0.0) + fps * c.pairs()
            s += 1
    return reqs, offered


def render_sources(classes: Sequence[ShapeClass], n_sources: int = 1, workers: int = 4):
    """Pre-render frames per class (seeded), in parallel processes."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    jobs = [(c.height, c.width, c.dtype, i) for c in classes for i in range(n_sources)]
    # fresh interpreters: the caller may already hold a GPU context
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=max(1, min(workers, len(jobs))), mp_context=ctx) as pool:
        frames = list(pool.map(_render_one, jobs))
    out = {}
    for (c, i), fr in zip([(c, i) for c in classes for i in range(n_sources)], frames):
        out.setdefault(c, []).append(fr)
    return {c: np.stack(v) for c, v in out.items()}


def _render_one(job):
    from paper_1706_07263_amd import synth
    h, w, dtype, i = job
    fr, _, _ = synth.single_frame(h, w, config=5, stream=100 + i + (h * 7 + w) % 97, dtype=dtype)
    return fr
