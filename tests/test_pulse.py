"""Temporal analysis (pulse detection) on THb traces: pins of each step on
signals with known answers, and the whole analysis on oracle estimates of a
small synthetic stereo video."""
import math

import numpy as np
import pytest

from oracle import hb_oracle as orc
from paper_1706_07263_amd import pulse, synth
from tests import hbtest

FPS = 30.0


def test_patch_series_ignores_nan():
    thb = np.arange(2 * 4 * 4, dtype=np.float64).reshape(2, 4, 4)
    thb[0, 1, 1] = np.nan
    s = pulse.patch_series(thb, (1, 3, 1, 3))
    assert s[0] == pytest.approx(np.mean([6, 9, 10]))
    assert s[1] == pytest.approx(np.mean([21, 22, 25, 26]))


def test_lowpass_response():
    """Constant passes unchanged; a sinusoid is scaled by the Gaussian's
    response exp(-(2 pi f s)^2 / 2), 1/sqrt(2) at the cutoff."""
    t = np.arange(600) / FPS
    assert np.allclose(pulse.lowpass(np.full(600, 3.5), FPS, 3.0), 3.5, rtol=0, atol=1e-12)
    sd = pulse.gaussian_sigma_s(3.0)
    assert math.exp(-(2 * math.pi * 3.0 * sd) ** 2 / 2) == pytest.approx(1 / math.sqrt(2))
    for f in (0.5, 1.25, 3.0, 6.0, 10.0):
        x = np.sin(2 * math.pi * f * t)
        y = pulse.lowpass(x, FPS, 3.0)
        gain = np.dot(y[100:500], x[100:500]) / np.dot(x[100:500], x[100:500])
        assert gain == pytest.approx(math.exp(-(2 * math.pi * f * sd) ** 2 / 2), abs=5e-3), f


def test_lowpass_is_zero_phase():
    t = np.arange(600) / FPS
    x = np.sin(2 * math.pi * 1.1 * t)
    y = pulse.lowpass(x, FPS, 3.0)
    g = np.dot(y[100:500], x[100:500]) / np.dot(x[100:500], x[100:500])
    assert np.max(np.abs(y[100:500] - g * x[100:500])) < 1e-9


def test_derivative_of_a_sinusoid():
    t = np.arange(300) / FPS
    x = np.sin(2 * math.pi * 1.25 * t)
    d = pulse.derivative(x, FPS)
    want = 2 * math.pi * 1.25 * np.cos(2 * math.pi * 1.25 * t)
    # central difference: sin(w h)/h instead of w, relative error (w h)^2/6
    h = 1 / FPS
    assert np.allclose(d[1:-1], want[1:-1] * math.sin(2 * math.pi * 1.25 * h) / (2 * math.pi * 1.25 * h),
                       rtol=0, atol=1e-12)


def test_derivative_of_a_quadratic_is_exact_inside():
    t = np.arange(50) / FPS
    d = pulse.derivative(3 * t ** 2 - t, FPS)
    assert np.allclose(d[1:-1], 6 * t[1:-1] - 1, rtol=0, atol=1e-10)


def test_quadratic_peak_refinement_is_exact_for_a_gaussian_line():
    """Log of a Gaussian line is a parabola: the three-point fit recovers its
    centre exactly, between bins."""
    f = np.linspace(0, 5, 101)
    for f0 in (1.2, 1.234, 2.01):
        p = np.exp(-((f - f0) / 0.3) ** 2)
        assert pulse.peak_frequency(f, p, (0.5, 4.0)) == pytest.approx(f0, abs=1e-9)


@pytest.mark.parametrize("f0", [1.17, 1.25, 1.31, 2.2])
def test_sinusoid_in_noise_is_located(f0):
    rng = np.random.default_rng(int(f0 * 100))
    t = np.arange(300) / FPS
    x = 100 + 2.0 * np.sin(2 * math.pi * f0 * t + 0.3) + rng.normal(0, 1.0, t.size) \
        + 3.0 * np.sin(2 * math.pi * 0.2 * t)
    a = pulse.analyse(x, FPS)
    assert a["peak_hz"] == pytest.approx(f0, abs=0.03)
    assert a["per_minute"] == pytest.approx(60 * a["peak_hz"])


def test_band_is_clipped_at_nyquist_and_aliasing():
    """Sampling a 2.2 Hz pulse at 3 frames/s (below 2 x 2.2) shows it at the
    alias 3 - 2.2 = 0.8 Hz; at 5 frames/s it is resolved."""
    assert pulse.min_frame_rate(2.0) == 4.0
    for fps, want in [(3.0, 0.8), (5.0, 2.2)]:
        t = np.arange(int(20 * fps)) / fps
        x = np.sin(2 * math.pi * 2.2 * t)
        a = pulse.analyse(x, fps, cutoff_hz=0.45 * fps, band=(0.5, 4.0))
        assert a["peak_hz"] == pytest.approx(want, abs=0.03)


def test_view_box_follows_the_shift():
    assert pulse.view_box((10, 20, 30, 40), 8.0, 0) == (10, 20, 30, 40)
    assert pulse.view_box((10, 20, 30, 40), 8.0, 1) == (10, 20, 22, 32)


def test_pulse_video_truth_and_views():
    spec = synth.PulseSpec(n_frames=4)
    v, thb = synth.pulse_video(16, 24, spec)
    assert v.shape == (2, 4, 16, 24, 3) and v.dtype == np.float32
    for f in range(4):
        assert np.allclose(thb[0, f], thb[0, 0] * synth.pulse_thb_factor(spec, f) /
                           synth.pulse_thb_factor(spec, 0))
    # the right view is the left field shifted by shift_px columns
    assert np.allclose(thb[1, 0, :, :16], thb[0, 0, :, 8:24])


def test_truth_trace_peaks_at_the_pulse():
    spec = synth.PulseSpec()
    _, thb = synth.pulse_video(16, 16, spec)
    for view in range(2):
        a = pulse.analyse(pulse.patch_series(thb[view], (4, 12, 4, 12)), spec.fps)
        assert a["peak_hz"] == pytest.approx(spec.pulse_hz, abs=0.02)


def test_oracle_estimates_resolve_the_pulse_in_both_views(spectra):
    """End to end on the CPU: oracle maps of a small noisy stereo video with
    roaming highlights; both views find the pulse and differ by a nearly
    constant offset (the right view's calibration mismatch)."""
    spec = synth.PulseSpec()
    h, w = 32, 48
    video, _ = synth.pulse_video(h, w, spec)
    s = synth.plan_settings(levels=1, grid=32)
    p = hbtest.oracle_params(w, h, s)
    m = hbtest.oracle_model(spectra)
    box = (8, 24, 16, 32)
    series = []
    for view in range(2):
        maps = orc.estimate(p, m, video[view].astype(np.float64))
        series.append(pulse.patch_series(maps[:, 2], pulse.view_box(box, spec.shift_px, view)))
    for x in series:
        assert pulse.analyse(x, spec.fps)["peak_hz"] == pytest.approx(spec.pulse_hz, abs=0.05)
    d = pulse.lowpass(series[1] - series[0], spec.fps, 0.5)
    assert abs(np.mean(d)) > 3 * np.std(d)
