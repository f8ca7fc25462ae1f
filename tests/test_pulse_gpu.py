"""Temporal workload on the GPU: THb of a tracked patch over a synthetic
stereo video, per-frame maps from the HIP path, pulse located in both views."""
import numpy as np
import pytest

from oracle import hb_oracle as orc
from paper_1706_07263_amd import pulse, synth
from tests import hbtest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_pulse_in_both_views(torch_cuda):
    spec = synth.PulseSpec()
    h, w = 96, 128
    video, thb_true = synth.pulse_video(h, w, spec)
    s = synth.plan_settings(levels=1, grid=64)
    box = (32, 64, 48, 80)
    p = hbtest.oracle_params(w, h, s)
    m = hbtest.oracle_model(synth.spectra())
    series = []
    for view in range(2):
        b = pulse.view_box(box, spec.shift_px, view)
        est = pulse.estimate_thb(video[view], s, b, batch=16)
        # parity of the patch THb on sampled frames
        for f in (0, 137, spec.n_frames - 1):
            ora = orc.estimate(p, m, video[view, f].astype(np.float64))[0, 2, b[0]:b[1], b[2]:b[3]]
            assert np.max(np.abs(est[f] - ora)) <= hbtest.TOL_THB, (view, f)
        x = pulse.patch_series(est, (0, b[1] - b[0], 0, b[3] - b[2]))
        a = pulse.analyse(x, spec.fps)
        t = pulse.analyse(pulse.patch_series(thb_true[view], b), spec.fps)
        print(f"view {view}: peak {a['peak_hz']:.4f} Hz ({a['per_minute']:.1f}/min), truth {t['peak_hz']:.4f} Hz,"
              f" mean THb {x.mean():.2f} uM")
        assert a["peak_hz"] == pytest.approx(spec.pulse_hz, abs=0.05)
        series.append(x)
    d = pulse.lowpass(series[1] - series[0], spec.fps, 0.5)
    assert abs(np.mean(d)) > 3 * np.std(d)
