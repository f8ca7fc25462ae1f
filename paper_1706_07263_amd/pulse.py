"""Temporal analysis of per-frame THb estimates: the pulse in a tracked patch.

Follows the paper's in vivo experiment (Experiments, Fig. 2): the mean THb
of a registered tissue patch is tracked over time in each view of a stereo
laparoscope, the trace is low-pass filtered (it carries much high-frequency
noise from specular highlights), differentiated, and the power spectrum of
the derivative peaks at the heart rate; a polynomial fitted around the peak
locates it between FFT bins.  The Conclusion adds that resolving a heart rate
above 2 Hz without aliasing needs more than 4 frames per second.

The per-frame estimates come from the GPU path (``hb.Plan``); the analysis
of the resulting 1-D series is a few hundred samples of host arithmetic.
"""
from __future__ import annotations

import argparse
import json
import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

Box = Tuple[int, int, int, int]   # rows [r0, r1), columns [c0, c1)


def patch_series(thb: np.ndarray, box: Box) -> np.ndarray:
    """Mean THb of the patch in every frame; thb [T][H][W]; NaN pixels ignored."""
    r0, r1, c0, c1 = box
    return np.nanmean(np.asarray(thb, dtype=np.float64)[:, r0:r1, c0:c1], axis=(1, 2))


def gaussian_sigma_s(cutoff_hz: float) -> float:
    """Time-domain s.d. (seconds) of the Gaussian whose response is 1/sqrt(2) at
    cutoff_hz: |H(f)| = exp(-(2 pi f s)^2 / 2)."""
    return math.sqrt(math.log(2.0)) / (2.0 * math.pi * cutoff_hz)


def lowpass(x: np.ndarray, fps: float, cutoff_hz: float) -> np.ndarray:
    """Zero-phase Gaussian low-pass filter (kernel truncated at 4 s.d.,
    edges mirrored)."""
    x = np.asarray(x, dtype=np.float64)
    sd = gaussian_sigma_s(cutoff_hz) * fps
    half = max(1, int(math.ceil(4.0 * sd)))
    t = np.arange(-half, half + 1, dtype=np.float64)
    k = np.exp(-0.5 * (t / sd) ** 2)
    k /= k.sum()
    if x.size <= half:
        raise ValueError("series shorter than the filter half-width")
    padded = np.concatenate([x[half:0:-1], x, x[-2:-half - 2:-1]])
    return np.convolve(padded, k, mode="valid")


def derivative(x: np.ndarray, fps: float) -> np.ndarray:
    """d/dt by central differences (one-sided at the ends), per second."""
    return np.gradient(np.asarray(x, dtype=np.float64)) * fps


def power_spectrum(x: np.ndarray, fps: float, pad: int = 8) -> Tuple[np.ndarray, np.ndarray]:
    """Hann-windowed power spectrum of the mean-removed series, zero-padded to
    pad x the next power of two."""
    x = np.asarray(x, dtype=np.float64)
    x = (x - x.mean()) * np.hanning(x.size)
    n = pad * (1 << int(math.ceil(math.log2(max(2, x.size)))))
    X = np.fft.rfft(x, n)
    return np.fft.rfftfreq(n, 1.0 / fps), np.abs(X) ** 2


def peak_frequency(freqs: np.ndarray, power: np.ndarray, band: Tuple[float, float]) -> float:
    """Frequency of the largest power inside band, refined by the vertex of a
    quadratic fitted to the log power at the peak and its two neighbours."""
    sel = np.nonzero((freqs >= band[0]) & (freqs <= band[1]))[0]
    if sel.size == 0:
        raise ValueError("no frequency bin inside the band")
    i = int(sel[np.argmax(power[sel])])
    if i == 0 or i == freqs.size - 1:
        return float(freqs[i])
    a, b, _ = np.polyfit(freqs[i - 1:i + 2] - freqs[i], np.log(power[i - 1:i + 2] + 1e-300), 2)
    if a >= 0:
        return float(freqs[i])
    return float(freqs[i] - b / (2.0 * a))


def min_frame_rate(heart_hz: float) -> float:
    """Sampling rate above which a heart rate of heart_hz does not alias."""
    return 2.0 * heart_hz


def analyse(series: np.ndarray, fps: float, cutoff_hz: float = 3.0,
            band: Tuple[float, float] = (0.5, 4.0)) -> Dict[str, object]:
    """Smooth, differentiate and locate the spectral peak of one THb trace."""
    if band[1] > 0.5 * fps:
        band = (band[0], 0.5 * fps)
    sm = lowpass(series, fps, cutoff_hz)
    d = derivative(sm, fps)
    f, p = power_spectrum(d, fps)
    pk = peak_frequency(f, p, band)
    return {"peak_hz": pk, "per_minute": 60.0 * pk, "smoothed": sm, "derivative": d,
            "freqs": f, "power": p}


def view_box(box: Box, shift_px: float, view: int) -> Box:
    """The same tissue patch in a view rendered with a horizontal shift."""
    s = int(round(view * shift_px))
    r0, r1, c0, c1 = box
    return (r0, r1, c0 - s, c1 - s)


def estimate_thb(frames: np.ndarray, settings: Dict[str, object], box: Box, dtype: str = "f32",
                 batch: int = 16, device: int = 0) -> np.ndarray:
    """Run the GPU path over frames [T][H][W][3] (storage dtype) in batches and
    return the patch's THb [T][r1-r0][c1-c0] (float64)."""
    import torch

    from . import hb
    from .synth import spectra
    T, H, W, _ = frames.shape
    r0, r1, c0, c1 = box
    desc = hb.make_desc(W, H, levels=int(settings["levels"]), dtype=dtype, max_batch=batch,
                        grid_thb=int(settings["grid_thb"]), grid_so2=int(settings["grid_so2"]),
                        thb_min=float(settings["thb_min"]), thb_max=float(settings["thb_max"]),
                        so2_min=float(settings["so2_min"]), so2_max=float(settings["so2_max"]),
                        lam=float(settings["lam"]), sigma=float(settings["sigma"]),
                        illumination=int(settings.get("illumination", 0)))
    out = np.empty((T, r1 - r0, c1 - c0))
    dev = torch.device("cuda", device)
    with hb.Plan(desc, device) as plan:
        plan.set_forward_model(spectra())
        thb = torch.empty((batch, H, W), device=dev, dtype=torch.float32)
        for t0 in range(0, T, batch):
            n = min(batch, T - t0)
            chunk = np.ascontiguousarray(frames[t0:t0 + n])
            src = torch.from_numpy(chunk.view(np.int16) if dtype == "bf16" else chunk).to(dev)
            plan.estimate(src, [None, None, thb[:n], None])
            out[t0:t0 + n] = thb[:n, r0:r1, c0:c1].double().cpu().numpy()
    return out


def main(argv: Optional[Sequence[str]] = None) -> None:
    from . import synth
    ap = argparse.ArgumentParser(description="pulse detection on a synthetic stereo video")
    ap.add_argument("--height", type=int, default=240)
    ap.add_argument("--width", type=int, default=320)
    ap.add_argument("--levels", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    args = ap.parse_args(argv)
    spec = synth.PulseSpec()
    video, thb_true = synth.pulse_video(args.height, args.width, spec)
    settings = synth.plan_settings(levels=args.levels, grid=args.grid)
    h, w = args.height, args.width
    box = (h // 2 - h // 8, h // 2 + h // 8, w // 2 - w // 8, w // 2 + w // 8)
    report = {"fps": spec.fps, "frames": spec.n_frames, "true_pulse_hz": spec.pulse_hz}
    for view in range(2):
        b = view_box(box, spec.shift_px, view)
        est = patch_series(estimate_thb(video[view], settings, b), (0, b[1] - b[0], 0, b[3] - b[2]))
        tru = patch_series(thb_true[view], b)
        a = analyse(est, spec.fps)
        report[f"view{view}"] = {"peak_hz": round(a["peak_hz"], 4), "per_minute": round(a["per_minute"], 2),
                                 "mean_thb_uM": round(float(est.mean()), 3),
                                 "truth_peak_hz": round(analyse(tru, spec.fps)["peak_hz"], 4)}
    print(json.dumps(report))


if __name__ == "__main__":
    main()
