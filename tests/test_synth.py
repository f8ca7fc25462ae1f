"""The seeded synthetic inputs: determinism, ranges and storage rounding."""
import numpy as np
import pytest
import torch

from paper_1706_07263_amd import synth


def test_fields_are_deterministic_and_in_range():
    a = synth.config1()
    b = synth.config1()
    assert np.array_equal(a.frames, b.frames)
    assert a.frames.shape == (1, 64, 64, 3) and a.frames.dtype == np.float32
    assert a.thb.min() >= 20.0 - 1e-9 and a.thb.max() <= 200.0 + 1e-9
    assert a.so2.min() >= 0.3 - 1e-12 and a.so2.max() <= 1.0 + 1e-12
    # both extremes of the normalised fields are reached on the reference canvas
    assert a.thb.min() == pytest.approx(20.0) and a.thb.max() == pytest.approx(200.0)
    assert 0.2 < a.frames.min() and a.frames.max() < 1.05


def test_noise_level():
    sp = synth.spectra()
    hb = np.full((256, 256), 40.0)
    hbo2 = np.full((256, 256), 60.0)
    clean = synth.render_intensity(hb, hbo2, sp)
    noisy = synth.noisy_frame(hb, hbo2, sp, 123).astype(np.float64)
    assert np.std(noisy - clean) == pytest.approx(synth.NOISE_SIGMA, rel=0.02)


def test_bf16_single_rounding_is_nearest():
    rng = np.random.default_rng(0)
    x = rng.uniform(0.01, 2.0, 20000)
    x = np.concatenate([x, [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0.5]])   # ties
    bits = synth.bf16_from_f64(x)
    v = synth.bf16_bits_to_f32(bits).astype(np.float64)
    for d in (-1, 1):
        nb = synth.bf16_bits_to_f32((bits.astype(np.int32) + d).astype(np.uint16)).astype(np.float64)
        assert np.all(np.abs(v - x) <= np.abs(nb - x))
    assert v[-3] == 1.0                      # tie 1 + 2^-8 rounds to even (1.0)
    assert v[-2] == 1.0 + 2.0 ** -6          # tie 1 + 3*2^-8 rounds to even
    # agrees with torch where the value is exactly representable in float32
    f = x.astype(np.float32)
    t = torch.from_numpy(f).to(torch.bfloat16).float().numpy()
    exact = f.astype(np.float64) == x
    assert np.array_equal(t[exact], v[exact].astype(np.float32))


def test_half_storage_is_exact_widening():
    w16 = synth.config1("f16")
    assert w16.frames.dtype == np.float16
    f64 = synth.storage_to_f64(w16.frames, "f16")
    assert np.array_equal(f64.astype(np.float16), w16.frames)


def test_stereo_views_share_the_scene():
    fr, thb, so2 = synth.stereo_pair(2, "f32", height=64, width=80, shift_px=16.0)
    assert fr.shape == (2, 64, 80, 3)
    assert np.allclose(thb[1][:, :-16], thb[0][:, 16:])


def test_video_motion_is_smooth():
    fr, thb, _ = synth.video_frames([0, 1, 150], height=72, width=128)
    d01 = np.abs(thb[1] - thb[0]).mean()
    d0150 = np.abs(thb[2] - thb[0]).mean()
    assert d01 < d0150


def test_serving_mix():
    streams = synth.serve_streams()
    assert len(streams) == 16
    mpx = sum(s.height * s.width * s.fps for s in streams) / 1e6
    assert mpx == pytest.approx(1019.9, rel=1e-3)
    t = synth.poisson_arrivals(3, 30.0, 20.0)
    assert 500 < t.size < 700 and np.all(np.diff(t) > 0)
