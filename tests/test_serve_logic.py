"""Serving logic on the CPU: admission by memory budget, continuous batching,
ordering, overlap of classes and failure handling (no GPU: FakeExecutor)."""
import math

import numpy as np
import pytest

from paper_1706_07263_amd.serve import FakeExecutor, FrameRequest, Server, ShapeClass, workload_requests

A = ShapeClass(64, 64, 1, 32)
B = ShapeClass(128, 128, 2, 64)
C = ShapeClass(256, 256, 2, 128)


def reqs_at(cls, times, stream=0):
    return [FrameRequest(stream=stream, index=i, cls=cls, arrival=t) for i, t in enumerate(times)]


def test_admission_respects_budget_and_refuses_what_does_not_fit():
    ex = FakeExecutor(cost=lambda c, b: 1e-3, lane_bytes=lambda c, b: {A: 100, B: 300, C: 1000}[c])
    srv = Server(ex, {A: 4, B: 4, C: 4}, hbm_budget=1000, offered={A: 1.0, B: 5.0, C: 0.5})
    assert srv.used <= 1000
    assert C in srv.refused                     # its first lane alone exceeds what is left
    # first lanes by load (B then A), then extra lanes round-robin while they fit
    assert [l.cls for l in srv.lanes[:3]] == [B, A, B]
    assert len(srv.by_class[B]) == 2 and len(srv.by_class[A]) == 4
    rep = srv.run(reqs_at(C, [0.0, 0.001]) + reqs_at(A, [0.0]))
    assert rep.failed == 2 and rep.frames == 1
    assert rep.refused == ["256x256/L2/G128/f16"]


def test_continuous_batching_takes_everything_that_arrived():
    cost = 0.02
    ex = FakeExecutor(cost=lambda c, b: cost)
    srv = Server(ex, {A: 8}, hbm_budget=10 ** 9, max_lanes=1)
    # one frame starts the lane; 5 more arrive while it is busy -> one batch of 5
    times = [0.0] + [0.005 + 0.001 * k for k in range(5)]
    rep = srv.run(reqs_at(A, times))
    sizes = [len(s[1]) for s in ex.submissions]
    assert sizes == [1, 5]
    assert rep.frames == 6 and rep.failed == 0
    assert rep.waited == 5
    lat = np.sort(rep.latencies_ms)
    assert lat[0] >= cost * 1e3 * 0.9
    assert lat[-1] <= 3 * cost * 1e3 + 20          # second batch waits for the first


def test_batches_are_bounded_and_fifo():
    ex = FakeExecutor(cost=lambda c, b: 0.01)
    srv = Server(ex, {A: 3}, hbm_budget=10 ** 9, max_lanes=1)
    rep = srv.run(reqs_at(A, [0.0] * 10))
    sizes = [len(s[1]) for s in ex.submissions]
    assert max(sizes) <= 3 and sum(sizes) == 10
    order = [idx for _, batch in ex.submissions for _, idx in batch]
    assert order == list(range(10))
    assert rep.frames == 10


def test_classes_overlap_on_their_own_lanes():
    cost = 0.05
    ex = FakeExecutor(cost=lambda c, b: cost)
    srv = Server(ex, {A: 1, B: 1}, hbm_budget=10 ** 9, max_lanes=1)
    rep = srv.run(reqs_at(A, [0.0]) + reqs_at(B, [0.0], stream=1))
    assert rep.frames == 2
    assert np.max(rep.latencies_ms) < 1.6 * cost * 1e3     # concurrent, not 2 x cost


def test_more_lanes_serve_more_concurrently():
    cost = 0.04
    ex = FakeExecutor(cost=lambda c, b: cost)
    one = Server(ex, {A: 1}, hbm_budget=10 ** 9, max_lanes=1).run(reqs_at(A, [0.0] * 4))
    ex2 = FakeExecutor(cost=lambda c, b: cost)
    four = Server(ex2, {A: 1}, hbm_budget=10 ** 9, max_lanes=4).run(reqs_at(A, [0.0] * 4))
    assert np.max(four.latencies_ms) < 0.5 * np.max(one.latencies_ms)


def test_failed_submission_fails_only_its_frames():
    bad = {"n": 0}

    def fail(lane, reqs):
        bad["n"] += 1
        return bad["n"] == 2

    ex = FakeExecutor(cost=lambda c, b: 0.005, fail=fail)
    srv = Server(ex, {A: 1}, hbm_budget=10 ** 9, max_lanes=1)
    rep = srv.run(reqs_at(A, [0.0, 0.02, 0.04]))
    assert rep.failed == 1 and rep.frames == 2


def test_warmup_window_and_summary():
    ex = FakeExecutor(cost=lambda c, b: 0.002 * b)
    srv = Server(ex, {A: 4, B: 2}, hbm_budget=10 ** 9)
    reqs = reqs_at(A, np.arange(0, 0.3, 0.01)) + reqs_at(B, np.arange(0, 0.3, 0.02), stream=1)
    rep = srv.run(reqs, warmup_s=0.1)
    s = rep.summary()
    assert s["frames"] == sum(1 for r in reqs if r.arrival >= 0.1)
    assert 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    assert set(s["per_class"]) == {"64x64/L1/G32/f16", "128x128/L2/G64/f16"}


def test_sixteen_stream_workload_shape():
    reqs, offered = workload_requests(2.0)
    streams = {r.stream for r in reqs}
    assert streams == set(range(16))
    assert 0.7 * 16 * 60 < len(reqs) < 1.3 * 16 * 60
    total = sum(offered.values())
    assert 2.0e12 < total < 3.5e12                      # posterior pairs per second offered
