"""Serving on the GPU: continuous batching over HIP-graph replays of the C-ABI
path; each served frame's maps equal (bitwise) the same frame run alone,
eagerly, through a fresh plan of its class."""
import numpy as np
import pytest

from paper_1706_07263_amd import synth
from paper_1706_07263_amd.serve import (FrameRequest, GpuExecutor, Server, ShapeClass, render_sources,
                                        workload_requests)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_mixed_streams_match_alone(torch_cuda):
    torch = torch_cuda
    classes = ((2, 128, 160, 1, 64), (2, 256, 320, 2, 128), (1, 96, 128, 1, 32))
    reqs, offered = workload_requests(1.5, classes=classes, fps=60.0, n_sources=2)
    cls = sorted(offered, key=lambda c: c.pixels)
    raw = render_sources(cls, n_sources=2, workers=2)
    sources = {c: torch.from_numpy(v).pin_memory() for c, v in raw.items()}
    keep = {(r.stream, r.index) for r in reqs[::7]}
    ex = GpuExecutor(synth.spectra(), sources, keep_outputs=lambda r: (r.stream, r.index) in keep)
    srv = Server(ex, {c: 4 for c in cls}, hbm_budget=8 << 30, offered=offered, max_lanes=2)
    rep = srv.run(reqs)
    s = rep.summary()
    print("serving summary", {k: v for k, v in s.items() if k != "per_class"})
    assert s["failed"] == 0 and s["frames"] == len(reqs)
    assert np.isfinite(s["p99_ms"])
    assert s["mean_batch"] >= 1.0
    by_key = {(r.stream, r.index): r for r in reqs}
    assert len(ex.kept) == len(keep)
    batched = 0
    for key, maps in ex.kept.items():
        r = by_key[key]
        alone = ex.run_alone(r.cls, r.source, max_batch=4)
        assert np.array_equal(maps, alone, equal_nan=True), key
        batched += r.batch > 1
    print("checked", len(ex.kept), "frames,", batched, "served inside a batch")
    srv.close()


def _burst_requests(classes, sizes, gap_s):
    """Bursts of frames that arrive at the same instant, one class at a time:
    a free lane takes the whole burst (up to its max batch), so every burst
    size is served as one batch of that size."""
    reqs = []
    t = 0.05
    stream = 0
    for c in classes:
        for size in sizes:
            for k in range(size):
                reqs.append(FrameRequest(stream=stream, index=k, cls=c, arrival=t, source=(stream + k) % 4))
            stream += 1
            t += gap_s
    return reqs


def test_every_batch_size_replayed_and_checked(torch_cuda):
    """Deterministic bursts make every class replay its captured graph at
    every batch size 1..4; every served frame equals (bitwise) the frame run
    alone, and one batched frame per class matches the FP64 oracle."""
    from tests import hbtest
    torch = torch_cuda
    spec = ((1, 128, 160, 1, 64), (1, 256, 320, 2, 128), (1, 96, 128, 1, 32))
    cls = [ShapeClass(h, w, lv, g, "f16") for _, h, w, lv, g in spec]
    raw = render_sources(cls, n_sources=4, workers=2)
    sources = {c: torch.from_numpy(v).pin_memory() for c, v in raw.items()}
    ex = GpuExecutor(synth.spectra(), sources, keep_outputs=lambda r: True)
    srv = Server(ex, {c: 4 for c in cls}, hbm_budget=8 << 30, max_lanes=1)
    reqs = _burst_requests(cls, (4, 3, 2, 1, 4), gap_s=0.25)
    rep = srv.run(reqs)
    s = rep.summary()
    assert s["failed"] == 0 and s["frames"] == len(reqs)
    for c in cls:
        served = {r.batch for r in reqs if r.cls == c}
        assert served == {1, 2, 3, 4}, (c, served)
    assert len(ex.kept) == len(reqs)
    by_key = {(r.stream, r.index): r for r in reqs}
    alone = {}
    for key, maps in ex.kept.items():
        r = by_key[key]
        if (r.cls, r.source) not in alone:
            alone[(r.cls, r.source)] = ex.run_alone(r.cls, r.source, max_batch=4)
        assert np.array_equal(maps, alone[(r.cls, r.source)], equal_nan=True), (key, r.batch)
    for c in cls:
        r = next(r for r in reqs if r.cls == c and r.batch == 4 and r.index == 3)
        settings = synth.plan_settings(levels=c.levels, grid=c.grid)
        ora = hbtest.run_oracle(raw[c][r.source][None], c.dtype, settings)
        err = hbtest.assert_maps_close(ex.kept[(r.stream, r.index)][None], ora, f"served {c} in a batch of 4")
        print("served frame vs oracle", c, {k: f"{v:.2e}" for k, v in err.items()})
    srv.close()
