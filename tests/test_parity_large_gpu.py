"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses.  The stereo pair and the video frames are compared with the
oracle on every pixel; the 512x512-grid and 3840x2160 cases, where the oracle
would take minutes per frame, on aligned crops (four corners plus random
interior crops), which reproduce the full-frame values because Haar blocks
are independent."""
import numpy as np
import pytest

from paper_1706_07263_amd import synth
from tests import hbtest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_stereo_pair_1280x1024(torch_cuda):
    w = synth.config2()
    run = hbtest.GpuRun(1280, 1024, w.plan, max_batch=2)
    gpu = run(w.frames)
    # both whole views against the oracle (every pixel)
    ora = hbtest.run_oracle(w.frames, "f32", w.plan)
    err = hbtest.assert_maps_close(gpu, ora, "stereo pair, whole views")
    print("stereo pair errors (whole views)", err)
    run.close()


def test_video_1920x1080_frames_0_150_299(torch_cuda):
    """The benchmark's launch: a plan for 16 frames and a full 16-frame call
    (the three frames repeated); the three whole frames against the oracle."""
    w = synth.config3((0, 150, 299))
    run = hbtest.GpuRun(1920, 1080, w.plan, max_batch=16)
    batch = np.ascontiguousarray(np.concatenate([w.frames] * 6)[:16])
    gpu = run(batch)
    # the three whole frames against the oracle (every pixel)
    ora = hbtest.run_oracle(w.frames, "f32", w.plan)
    err = hbtest.assert_maps_close(gpu[:3], ora, "video frames 0/150/299, whole frames")
    print("video errors (whole frames)", err)
    # every repeat of a frame inside the batch, and the frame alone, give the same bits
    for i in range(3, 16):
        assert np.array_equal(gpu[i], gpu[i % 3], equal_nan=True), i
    alone = run(w.frames[1:2])
    assert np.array_equal(alone[0], gpu[1], equal_nan=True)
    run.close()


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_half_storage_grid_512(torch_cuda, dtype):
    w = synth.config4(dtype)
    run = hbtest.GpuRun(1280, 1024, w.plan, dtype=dtype, max_batch=2)
    gpu = run(w.frames)
    err = hbtest.sampled_parity(gpu, w.frames, dtype, w.plan, hbtest.crops(1024, 1280, 1, 16, 8, 4), where=dtype)
    print(dtype, "errors vs oracle on the stored input", err)
    run.close()


def test_largest_frame_3840x2160(torch_cuda):
    fr, _, _ = synth.single_frame(2160, 3840, config=5, stream=14, dtype="f16")
    s = synth.plan_settings(levels=2, grid=128)
    run = hbtest.GpuRun(3840, 2160, s, dtype="f16")
    gpu = run(fr[None])
    hbtest.sampled_parity(gpu, fr[None], "f16", s, hbtest.crops(2160, 3840, 2, 32, 8, 5), where="4k")
    run.close()


U_ROUND = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def _posterior_jacobian(c, mu, ybar, sigma, h=1e-6):
    from oracle import hb_oracle as orc
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (orc.posterior_mean(c, mu, ybar + e, sigma) - orc.posterior_mean(c, mu, ybar - e, sigma)) / (2 * h)
    return J


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_half_storage_error_bound_vs_unquantised(torch_cuda, dtype):
    """Half-precision storage against the oracle on the unquantised (FP32)
    frames.  Rounding each intensity changes its log-attenuation by at most
    u (unit roundoff of the storage type), so per pixel
        |dc| <= u (||J_post||_inf + 2 ||M||_inf) + 1e-4 uM,
    with J_post the oracle posterior mean's Jacobian at the pixel's block
    (central differences) and M the Tikhonov operator."""
    from oracle import hb_oracle as orc
    w16 = synth.config4(dtype)
    f32, _, _ = synth.stereo_pair(2, "f32")
    s = w16.plan
    run = hbtest.GpuRun(1280, 1024, s, dtype=dtype, max_batch=2)
    gpu = run(w16.frames)
    Mi = np.abs(run.plan.info()["M"]).sum(axis=1).max()
    run.close()
    model = hbtest.oracle_model(synth.spectra())
    cg, mug = orc.grid(hbtest.oracle_params(16, 16, s), model)
    u = U_ROUND[dtype]
    worst_ratio, errs = 0.0, {k: [] for k in ("hb", "hbo2", "so2")}
    for (r, c, hh, ww) in hbtest.crops(1024, 1280, 1, 16, 6, 7):
        sub = np.ascontiguousarray(f32[:, r:r + hh, c:c + ww])
        ora = hbtest.run_oracle(sub, "f32", s)
        g = gpu[:, :, r:r + hh, c:c + ww].astype(np.float64)
        y = -np.log(np.maximum(sub.astype(np.float64), 1e-4))
        ybar = y.reshape(2, hh // 2, 2, ww // 2, 2, 3).mean(axis=(2, 4))
        for v in range(2):
            for bi in range(hh // 2):
                for bj in range(ww // 2):
                    J = _posterior_jacobian(cg, mug, ybar[v, bi, bj], s["sigma"])
                    bound = u * (np.abs(J).sum(axis=1).max() + 2 * Mi) + 1e-4
                    blk = (slice(2 * bi, 2 * bi + 2), slice(2 * bj, 2 * bj + 2))
                    d = np.abs(g[v, :2][(slice(None),) + blk] - ora[v, :2][(slice(None),) + blk]).max()
                    worst_ratio = max(worst_ratio, d / bound)
        errs["hb"].append(np.abs(g[:, 0] - ora[:, 0]).ravel())
        errs["hbo2"].append(np.abs(g[:, 1] - ora[:, 1]).ravel())
        m = ora[:, 2] >= 1.0
        errs["so2"].append(np.abs(g[:, 3] - ora[:, 3])[m].ravel())
    stats = {k: (float(np.concatenate(v).max()), float(np.sqrt(np.mean(np.concatenate(v) ** 2)))) for k, v in errs.items()}
    print(dtype, "vs unquantised: max/RMS", stats, "worst |dc|/bound", worst_ratio)
    assert worst_ratio <= 1.0
