"""The allocation-free estimate call against hb_estimate_frames, through the C
ABI: hb_estimate_frames_noalloc keeps the call's intermediate buffers in the
library's static per-device scratch array and must give the same maps, bit
for bit (same kernels, same arithmetic), on two calls in a row, the second
with fewer frames than the first (the scratch keeps the first call's
contents).  Cases cover the fused path (one grid split, MFMA posterior,
maps written by the posterior), split grids (global reference, partials and
the merge kernel in the scratch), the direct posterior with three levels
(LDS Haar kernel and recomposition), the Tikhonov low-pass (no partials),
a call near the array's capacity, and the host-side refusal of a call that
does not fit."""
import numpy as np
import pytest

from paper_1706_07263_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _frames(n, h, w, seed_stream):
    fr = [synth.single_frame(h, w, config=7, stream=seed_stream, frame=i)[0] for i in range(n)]
    return np.stack(fr)


def _maps(torch, n, h, w):
    return [torch.full((n, h, w), float("nan"), device="cuda", dtype=torch.float32) for _ in range(4)]


def _both(torch, plan, d, h, w):
    n = d.shape[0]
    ref, got = _maps(torch, n, h, w), _maps(torch, n, h, w)
    plan.estimate(d, ref)
    plan.estimate(d, got, noalloc=True)
    torch.cuda.synchronize()
    return (np.stack([m.cpu().numpy() for m in ref], 1), np.stack([m.cpu().numpy() for m in got], 1))


CASES = [
    # (h, w, levels, grid, sigma, split, lowpass, n_first, n_second)
    (480, 640, 2, 256, 0.01, 0, 0, 4, 2),     # fused: one split, MFMA, maps from the posterior
    (192, 256, 1, 64, 0.01, 3, 0, 3, 1),      # split grid: K2a reference, partials, K3 merge
    (128, 128, 3, 48, 1e-3, 0, 0, 3, 1),      # direct posterior, LDS Haar, K3
    (192, 256, 2, 64, 0.01, 0, 1, 3, 2),      # Tikhonov low-pass: no partials
]


@pytest.mark.parametrize("h,w,levels,grid,sigma,split,lowpass,n1,n2", CASES)
def test_noalloc_equals_plan_scratch_twice(torch_cuda, h, w, levels, grid, sigma, split, lowpass, n1, n2):
    torch = torch_cuda
    from paper_1706_07263_amd import hb
    print(f"noalloc case {h}x{w} L{levels} G{grid} sigma {sigma} split {split} lowpass {lowpass}", flush=True)
    desc = hb.make_desc(w, h, levels=levels, max_batch=max(n1, n2), grid_thb=grid, grid_so2=grid,
                        sigma=sigma, grid_split=split, lowpass=lowpass)
    frames = _frames(n1 + n2, h, w, seed_stream=levels)
    with hb.Plan(desc, 0) as plan:
        plan.set_forward_model(synth.spectra())
        info = plan.info()
        print("plan", info["posterior_kernel"], "split", info["grid_split"], flush=True)
        if split:
            assert info["grid_split"] == split
        for sel in (slice(0, n1), slice(n1, n1 + n2)):
            d = torch.from_numpy(np.ascontiguousarray(frames[sel])).cuda()
            ref, got = _both(torch, plan, d, h, w)
            assert np.isfinite(ref[:, :3]).all()
            assert np.array_equal(ref, got, equal_nan=True), f"frames {sel}"


def test_noalloc_near_capacity_then_smaller(torch_cuda):
    torch = torch_cuda
    from paper_1706_07263_amd import hb
    h, w = 1080, 1920
    # 1920x1080, 2 levels, one split: 23.8 MB of call buffers per frame; 5 fit in 128 MiB.
    print("noalloc case 1920x1080 L2 G256, 5 frames then 2", flush=True)
    fr, _, _ = synth.video_frames([0, 75, 150, 225, 299])
    desc = hb.make_desc(w, h, levels=2, max_batch=5, grid_thb=256, grid_so2=256)
    with hb.Plan(desc, 0) as plan:
        plan.set_forward_model(synth.spectra())
        # second call: two frames, in slots that held other frames in the first
        for sel in ([0, 1, 2, 3, 4], [4, 1]):
            d = torch.from_numpy(np.ascontiguousarray(fr[sel])).cuda()
            ref, got = _both(torch, plan, d, h, w)
            assert np.array_equal(ref, got, equal_nan=True), f"frames {sel}"


def test_noalloc_refuses_calls_beyond_the_scratch(torch_cuda):
    torch = torch_cuda
    from paper_1706_07263_amd import hb
    # 3840x2160 at one level: 182 MB of call buffers for one frame.
    h, w = 2160, 3840
    desc = hb.make_desc(w, h, levels=1, max_batch=1, grid_thb=16, grid_so2=16)
    with hb.Plan(desc, 0) as plan:
        plan.set_forward_model(synth.spectra())
        d = torch.full((1, h, w, 3), 0.5, device="cuda", dtype=torch.float32)
        maps = _maps(torch, 1, h, w)
        with pytest.raises(hb.HbError) as e:
            plan.estimate(d, maps, noalloc=True)
        assert e.value.status == hb.HB_ERR_SCRATCH
        torch.cuda.synchronize()
        assert all(torch.isnan(m).all().item() for m in maps)   # nothing was launched
        plan.estimate(d, maps)                                   # the plan's own scratch still works
        torch.cuda.synchronize()
        assert all(torch.isfinite(m[:, :8, :8]).all().item() for m in maps[:3])


def test_noalloc_inside_a_captured_graph(torch_cuda):
    """The call's use case: captured into a HIP graph (nothing to allocate
    during capture), then replayed on new inputs with eager work between the
    replays; every replay equals the eager call on the same frames."""
    torch = torch_cuda
    from paper_1706_07263_amd import hb
    h, w = 192, 256
    print("noalloc graph case 256x192 L2 G64, batch 2", flush=True)
    desc = hb.make_desc(w, h, levels=2, max_batch=2, grid_thb=64, grid_so2=64)
    sets = [np.ascontiguousarray(_frames(2, h, w, seed_stream=40 + k)) for k in range(3)]
    with hb.Plan(desc, 0) as plan:
        plan.set_forward_model(synth.spectra())
        stream = torch.cuda.Stream()
        inp = torch.zeros((2, h, w, 3), device="cuda", dtype=torch.float32)
        out = _maps(torch, 2, h, w)
        with torch.cuda.stream(stream):
            plan.estimate(inp, out, stream, noalloc=True)      # warm-up outside the capture
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            plan.estimate(inp, out, stream, noalloc=True)
        stream.synchronize()
        for k in (0, 1, 2, 0):
            inp.copy_(torch.from_numpy(sets[k]))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = np.stack([m.cpu().numpy() for m in out], 1)
            ref = _maps(torch, 2, h, w)
            plan.estimate(torch.from_numpy(sets[k]).cuda(), ref)    # eager, the plan's own scratch
            torch.cuda.synchronize()
            want = np.stack([m.cpu().numpy() for m in ref], 1)
            assert np.array_equal(got, want, equal_nan=True), f"replay of set {k}"
        del g
