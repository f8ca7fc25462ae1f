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
