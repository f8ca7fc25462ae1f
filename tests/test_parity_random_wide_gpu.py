"""GPU parity on seeded random configurations over wider ranges than the
standard set: frame sizes up to 192 (ragged against the 8-pixel tiles), Haar
levels 0-5, non-square grids of 1 to 160 nodes per axis over THb ranges from
1-60 to 100-400 uM and SO2 from 0-0.5 to 0.7-1, likelihood sigma 0.002 to
0.05 (at 0.002, observations of noisy half-precision frames lie tens of
scaled units from the nearest node), Tikhonov lambda 1e-5 to 1e-1, both
low-pass modes, the illumination term, the three skipping modes, forced grid
splits, FP32/FP16/BF16 storage, batches of 1-3 frames and the three cameras,
each against the FP64 oracle at every pixel."""
import numpy as np
import pytest

from paper_1706_07263_amd import synth
from tests import hbtest

pytestmark = pytest.mark.gpu

N_CASES = 300


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def random_case(seed: int):
    rng = np.random.default_rng(77000 + seed)
    levels = int(rng.integers(0, 6))
    b = 1 << levels
    h = int(rng.integers(max(1, 8 // b), 192 // b + 1)) * b
    w = int(rng.integers(max(1, 8 // b), 192 // b + 1)) * b
    thb_min = float(rng.uniform(1.0, 60.0))
    so2_min = float(rng.uniform(0.0, 0.5))
    s = dict(levels=levels, grid_thb=int(rng.integers(1, 161)), grid_so2=int(rng.integers(1, 161)),
             thb_min=thb_min, thb_max=float(rng.uniform(100.0, 400.0)),
             so2_min=so2_min, so2_max=float(rng.uniform(0.7, 1.0)),
             lam=float(10.0 ** rng.uniform(-5, -1)), sigma=float(rng.choice([0.002, 0.004, 0.006, 0.01, 0.02, 0.05])),
             illumination=int(rng.random() < 0.25),
             posterior_tolerance=float(rng.choice([1e-6, 1e-6, 1e-5, 0.0, -1.0])))
    lowpass = int(rng.random() < 0.15)
    split = int(rng.choice([0, 0, 0, 2, 5]))
    dtype = str(rng.choice(["f32", "f32", "f16", "bf16"]))
    n = int(rng.integers(1, 4))
    camera = str(rng.choice(["default", "default", "shifted", "narrow"]))
    return h, w, s, lowpass, split, dtype, n, camera


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_configuration(torch_cuda, seed):
    h, w, s, lowpass, split, dtype, n, camera = random_case(seed)
    sp = synth.spectra() if camera == "default" else synth.alt_spectra(camera)
    frames = np.stack([synth.single_frame(h, w, config=90, stream=seed, frame=i, dtype=dtype, sp=sp)[0]
                       for i in range(n)])
    where = (f"seed {seed}: {h}x{w} L{s['levels']} G{s['grid_thb']}x{s['grid_so2']} sigma {s['sigma']} "
             f"lowpass {lowpass} illum {s['illumination']} tol {s['posterior_tolerance']} split {split} "
             f"{dtype} n {n} camera {camera}")
    print(where, flush=True)
    run = hbtest.GpuRun(w, h, s, dtype=dtype, max_batch=n, lowpass=lowpass, grid_split=split, sp=sp)
    info = run.plan.info()
    run.hb.hb_plan_set_timing(run.plan.handle, True)
    gpu = run(frames)
    far = run.hb.hb_plan_get_far_pixels(run.plan.handle)
    run.close()
    ora = hbtest.run_oracle(frames, dtype, s, lowpass=lowpass, sp=sp)
    err = hbtest.assert_maps_close(gpu, ora, where)
    print("  kernel", info["posterior_kernel"], "split", info["grid_split"], "R2h", f"{info['mfma_index']:.0f}",
          "far pixels", far,
          {k: f"{v:.2e}" for k, v in err.items()})
