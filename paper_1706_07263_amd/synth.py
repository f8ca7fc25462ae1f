"""Seeded synthetic inputs for the haemoglobin-estimation path.

This module is the *world*: it draws ground-truth haemoglobin fields, renders
RGB frames from them through Beer-Lambert absorption integrated over the camera
responses, adds sensor noise and quantises to the storage dtype.  It holds none
of the estimation method's arithmetic (no log-attenuation, no Haar transform,
no inversion, no posterior); both the FP64 oracle and the GPU path receive the
arrays it returns as plain inputs.

The paper evaluates on in vivo multispectral data and on a stereo laparoscope
video that are not available here (Experiments, sections 3.1 and 3.2).  The
generators below stand in for them with frames of the same kind: mega-pixel RGB
frames of smooth tissue-like haemoglobin fields, a stereo pair, and a moving
video.  Every draw is seeded: ``seed = 1000*config + 10*stream + field_id`` for
fields and ``seed + frame_index`` (on a separate stream) for noise.

Spectral model (a proposal, not the paper's data): wavelengths 400..700 nm at
5 nm; extinction curves of HbO2 and Hb in natural-log units (cm^-1 uM^-1), each
a sum of three Gaussians (Soret-like peak near 420 nm and two Q-bands near
540/575 nm); camera responses are Gaussians at 460/540/610 nm with sigma 30 nm;
path length 0.1 cm; intensity noise sigma 0.005.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

WAVELENGTHS_NM = np.arange(400.0, 701.0, 5.0)
# (amplitude cm^-1 uM^-1, centre nm, sigma nm)
EPS_HBO2_TERMS = ((1.0, 418.0, 15.0), (0.06, 542.0, 10.0), (0.065, 577.0, 9.0))
EPS_HB_TERMS = ((0.8, 432.0, 18.0), (0.055, 550.0, 20.0), (0.04, 575.0, 45.0))
RESPONSE_TERMS = ((460.0, 30.0), (540.0, 30.0), (610.0, 30.0))  # R, G, B order below
PATH_LENGTH_CM = 0.1
NOISE_SIGMA = 0.005
THB_RANGE = (20.0, 200.0)   # uM
SO2_RANGE = (0.3, 1.0)      # fraction


@dataclasses.dataclass(frozen=True)
class Spectra:
    wavelength_nm: np.ndarray   # [n]
    eps_hb: np.ndarray          # [n] cm^-1 uM^-1, natural log
    eps_hbo2: np.ndarray        # [n]
    response: np.ndarray        # [3][n]  R, G, B (unnormalised)
    path_length_cm: float


def _gauss_sum(x: np.ndarray, terms) -> np.ndarray:
    out = np.zeros_like(x, dtype=np.float64)
    for amp, mu, sd in terms:
        out += amp * np.exp(-0.5 * ((x - mu) / sd) ** 2)
    return out


def spectra() -> Spectra:
    wl = WAVELENGTHS_NM.copy()
    # Camera channels ordered R, G, B: 610, 540, 460 nm.
    resp = np.stack([_gauss_sum(wl, ((1.0, c, s),)) for (c, s) in reversed(RESPONSE_TERMS)])
    return Spectra(wl, _gauss_sum(wl, EPS_HB_TERMS), _gauss_sum(wl, EPS_HBO2_TERMS), resp,
                   PATH_LENGTH_CM)


# Other cameras for tests of the forward-model handling: the same extinction
# curves with different channel responses and path length.
#   "shifted": responses moved by 20 nm (R 630, G 520, B 480 nm) and a 0.2 cm
#              path (cond(E) 10.6 at the grid centre, |M|_inf 1.4e3);
#   "narrow":  responses 600/560/520 nm, 0.2 cm (closely spaced channels,
#              cond(E) 14.8, |M|_inf 1.4e3).
ALT_CAMERAS = {"shifted": ((630.0, 520.0, 480.0), 0.2), "narrow": ((600.0, 560.0, 520.0), 0.2)}


def alt_spectra(name: str) -> Spectra:
    centres, path = ALT_CAMERAS[name]
    wl = WAVELENGTHS_NM.copy()
    resp = np.stack([_gauss_sum(wl, ((1.0, c, 30.0),)) for c in centres])
    return Spectra(wl, _gauss_sum(wl, EPS_HB_TERMS), _gauss_sum(wl, EPS_HBO2_TERMS), resp, path)


# ----------------------------------------------------------------------------
# Ground-truth fields: sums of Gaussian blobs, analytic so they can be sampled
# at moved coordinates.
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class BlobField:
    cy: np.ndarray
    cx: np.ndarray
    sd: np.ndarray
    amp: np.ndarray
    lo: float   # min over the reference canvas
    hi: float   # max over the reference canvas

    def raw(self, yy: np.ndarray, xx: np.ndarray) -> np.ndarray:
        out = np.zeros(np.broadcast(yy, xx).shape, dtype=np.float64)
        for cy, cx, sd, a in zip(self.cy, self.cx, self.sd, self.amp):
            out += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * sd * sd))
        return out

    def unit(self, yy: np.ndarray, xx: np.ndarray) -> np.ndarray:
        return np.clip((self.raw(yy, xx) - self.lo) / (self.hi - self.lo), 0.0, 1.0)


def make_blob_field(height: int, width: int, seed: int, n_blobs: int = 8) -> BlobField:
    rng = np.random.default_rng(seed)
    m = min(height, width)
    cy = rng.uniform(0, height, n_blobs)
    cx = rng.uniform(0, width, n_blobs)
    sd = rng.uniform(0.08, 0.25, n_blobs) * m
    amp = rng.uniform(0.3, 1.0, n_blobs)
    f = BlobField(cy, cx, sd, amp, 0.0, 1.0)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    r = f.raw(yy, xx)
    return dataclasses.replace(f, lo=float(r.min()), hi=float(r.max()))


@dataclasses.dataclass(frozen=True)
class Motion:
    """Smooth rigid motion: each of theta, tx, ty is a sum of 3 sinusoids."""
    freqs: np.ndarray    # [3][3] Hz
    phases: np.ndarray   # [3][3]
    amps: np.ndarray     # [3][3]
    fps: float

    def at(self, frame: int) -> Tuple[float, float, float]:
        t = frame / self.fps
        v = (self.amps * np.sin(2 * math.pi * self.freqs * t + self.phases)).sum(axis=1)
        return float(v[0]), float(v[1]), float(v[2])


def make_motion(seed: int, width: int, fps: float = 30.0) -> Motion:
    rng = np.random.default_rng(seed)
    freqs = rng.uniform(0.05, 0.5, (3, 3))
    phases = rng.uniform(0, 2 * math.pi, (3, 3))
    w = rng.uniform(0.2, 1.0, (3, 3))
    w /= w.sum(axis=1, keepdims=True)           # each component's amplitude sums to its cap
    caps = np.array([math.radians(10.0), 0.05 * width, 0.05 * width])
    return Motion(freqs, phases, w * caps[:, None], fps)


def truth(height: int, width: int, thb_field: BlobField, so2_field: BlobField,
          motion: Optional[Motion] = None, frame: int = 0, shift_x: float = 0.0
          ) -> Tuple[np.ndarray, np.ndarray]:
    """THb (uM) and SO2 (fraction) on the pixel grid of one frame."""
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    xx = xx + shift_x
    if motion is not None:
        th, tx, ty = motion.at(frame)
        cy, cx = 0.5 * (height - 1), 0.5 * (width - 1)
        c, s = math.cos(th), math.sin(th)
        dy, dx = yy - cy, xx - cx
        yy = cy + c * dy - s * dx - ty
        xx = cx + s * dy + c * dx - tx
    thb = THB_RANGE[0] + (THB_RANGE[1] - THB_RANGE[0]) * thb_field.unit(yy, xx)
    so2 = SO2_RANGE[0] + (SO2_RANGE[1] - SO2_RANGE[0]) * so2_field.unit(yy, xx)
    return thb, so2


# ----------------------------------------------------------------------------
# Image formation (the world model) and storage quantisation.
# ----------------------------------------------------------------------------

def render_intensity(hb: np.ndarray, hbo2: np.ndarray, sp: Spectra, chunk: int = 1 << 17
                     ) -> np.ndarray:
    """Noise-free RGB intensities [..., 3] in float64 by Beer-Lambert absorption
    integrated over each camera response (responses normalised to unit sum)."""
    resp = sp.response / sp.response.sum(axis=1, keepdims=True)      # [3][n]
    shape = np.broadcast(hb, hbo2).shape
    hb_f = np.broadcast_to(hb, shape).reshape(-1)
    hbo2_f = np.broadcast_to(hbo2, shape).reshape(-1)
    out = np.empty((hb_f.size, 3), dtype=np.float64)
    L = sp.path_length_cm
    for s in range(0, hb_f.size, chunk):
        e = slice(s, min(s + chunk, hb_f.size))
        att = np.exp(-L * (np.outer(hb_f[e], sp.eps_hb) + np.outer(hbo2_f[e], sp.eps_hbo2)))
        out[e] = att @ resp.T
    return out.reshape(shape + (3,))


def bf16_bits_rne(x: np.ndarray) -> np.ndarray:
    """float -> bfloat16 bit patterns (uint16), round-to-nearest-even; NaN kept NaN."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    nan = np.isnan(f)
    out = rounded.astype(np.uint16)
    out[nan] = 0x7FC0
    return out


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def quantise(x: np.ndarray, dtype: str) -> np.ndarray:
    """Cast float64 intensities to the storage dtype with round-to-nearest-even.
    'f32' -> float32, 'f16' -> float16, 'bf16' -> uint16 bit patterns."""
    if dtype == "f32":
        return np.ascontiguousarray(x, dtype=np.float32)
    if dtype == "f16":
        return np.ascontiguousarray(x, dtype=np.float16)
    if dtype == "bf16":
        # float64 -> float32 (RNE) -> bfloat16 (RNE) can double-round; go via the
        # exact float64 value instead.
        return bf16_from_f64(x)
    raise ValueError(dtype)


def bf16_from_f64(x: np.ndarray) -> np.ndarray:
    """float64 -> bfloat16 bits with a single round-to-nearest-even."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = x.astype(np.float32)                                  # may round
    b = bf16_bits_rne(f)
    # Correct double rounding: candidates b and its neighbours, pick nearest to x
    # (ties to even mantissa).
    out = b.copy()
    finite = np.isfinite(x)
    for d in (-1, 1):
        nb = (b.astype(np.int32) + d).astype(np.uint16)
        cur = np.abs(bf16_bits_to_f32(out).astype(np.float64) - x)
        alt = np.abs(bf16_bits_to_f32(nb).astype(np.float64) - x)
        better = finite & ((alt < cur) | ((alt == cur) & ((nb & 1) == 0) & ((out & 1) == 1)))
        out = np.where(better, nb, out)
    return out


def storage_to_f64(frames: np.ndarray, dtype: str) -> np.ndarray:
    """Exact widening of stored frames to float64."""
    if dtype == "bf16":
        return bf16_bits_to_f32(frames).astype(np.float64)
    return np.asarray(frames).astype(np.float64)


def noisy_frame(hb: np.ndarray, hbo2: np.ndarray, sp: Spectra, noise_seed: int,
                dtype: str = "f32", noise_sigma: float = NOISE_SIGMA) -> np.ndarray:
    clean = render_intensity(hb, hbo2, sp)
    rng = np.random.default_rng(noise_seed)
    noisy = clean + rng.normal(0.0, noise_sigma, clean.shape)
    return quantise(noisy, dtype)


def hb_hbo2(thb: np.ndarray, so2: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    return thb * (1.0 - so2), thb * so2


# ----------------------------------------------------------------------------
# Workloads.  Each returns frames [N][H][W][3] in the storage dtype plus the
# ground truth and the estimation settings the workload is defined with.
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    frames: np.ndarray                 # [N][H][W][3] storage dtype
    dtype: str                         # 'f32' | 'f16' | 'bf16'
    thb: np.ndarray                    # [N][H][W] ground truth (uM)
    so2: np.ndarray                    # [N][H][W]
    plan: Dict[str, object]            # estimation settings (levels, grid, lambda, sigma)


def _seed(config: int, stream: int, field_id: int) -> int:
    return 1000 * config + 10 * stream + field_id


def illumination_gain(height: int, width: int, seed: int, lo: float = 0.7, hi: float = 1.15
                      ) -> np.ndarray:
    """Smooth multiplicative illumination field [H][W][1] in [lo, hi]: the same
    gain on every colour channel of a pixel (a global-illumination change)."""
    f = make_blob_field(height, width, seed, n_blobs=4)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    return (lo + (hi - lo) * f.unit(yy, xx))[..., None]


def plan_settings(levels: int, grid: int, lam: float = 1e-3, sigma: float = 0.01) -> Dict[str, object]:
    return dict(levels=levels, grid_thb=grid, grid_so2=grid, thb_min=THB_RANGE[0],
                thb_max=THB_RANGE[1], so2_min=SO2_RANGE[0], so2_max=SO2_RANGE[1],
                lam=lam, sigma=sigma)


def single_frame(height: int = 64, width: int = 64, config: int = 1, stream: int = 0,
                 frame: int = 0, dtype: str = "f32", sp: Optional[Spectra] = None
                 ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    sp = sp or spectra()
    ft = make_blob_field(height, width, _seed(config, stream, 1))
    fs = make_blob_field(height, width, _seed(config, stream, 2))
    thb, so2 = truth(height, width, ft, fs)
    hb, hbo2 = hb_hbo2(thb, so2)
    fr = noisy_frame(hb, hbo2, sp, _seed(config, stream, 3) + frame, dtype)
    return fr, thb, so2


def config1(dtype: str = "f32") -> Workload:
    fr, thb, so2 = single_frame(64, 64, config=1, dtype=dtype)
    return Workload("single 64x64 frame", fr[None], dtype, thb[None], so2[None],
                    plan_settings(levels=1, grid=32))


def stereo_pair(config: int, dtype: str, height: int = 1024, width: int = 1280,
                shift_px: float = 16.0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    sp = spectra()
    ft = make_blob_field(height, width, _seed(config, 0, 1))
    fs = make_blob_field(height, width, _seed(config, 0, 2))
    frames, thbs, so2s = [], [], []
    for view, shift in enumerate((0.0, shift_px)):
        thb, so2 = truth(height, width, ft, fs, shift_x=shift)
        hb, hbo2 = hb_hbo2(thb, so2)
        frames.append(noisy_frame(hb, hbo2, sp, _seed(config, view, 3), dtype))
        thbs.append(thb)
        so2s.append(so2)
    return np.stack(frames), np.stack(thbs), np.stack(so2s)


def config2(dtype: str = "f32") -> Workload:
    fr, thb, so2 = stereo_pair(2, dtype)
    return Workload("stereo pair 1280x1024", fr, dtype, thb, so2, plan_settings(levels=1, grid=128))


def config4(dtype: str = "f16") -> Workload:
    # Same scene and noise draws as the stereo pair, stored in half precision.
    fr, thb, so2 = stereo_pair(2, dtype)
    return Workload(f"stereo pair 1280x1024 {dtype}", fr, dtype, thb, so2,
                    plan_settings(levels=1, grid=512))


def video_frames(frame_indices: Sequence[int], height: int = 1080, width: int = 1920,
                 config: int = 3, stream: int = 0, dtype: str = "f32"
                 ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    sp = spectra()
    ft = make_blob_field(height, width, _seed(config, stream, 1))
    fs = make_blob_field(height, width, _seed(config, stream, 2))
    mo = make_motion(_seed(config, stream, 4), width)
    frames, thbs, so2s = [], [], []
    for f in frame_indices:
        thb, so2 = truth(height, width, ft, fs, motion=mo, frame=f)
        hb, hbo2 = hb_hbo2(thb, so2)
        frames.append(noisy_frame(hb, hbo2, sp, _seed(config, stream, 3) + f, dtype))
        thbs.append(thb)
        so2s.append(so2)
    return np.stack(frames), np.stack(thbs), np.stack(so2s)


def config3(frame_indices: Sequence[int] = (0,), dtype: str = "f32") -> Workload:
    fr, thb, so2 = video_frames(frame_indices, dtype=dtype)
    return Workload("1920x1080 video", fr, dtype, thb, so2, plan_settings(levels=2, grid=256))


# Temporal workload: a registered stereo video of tissue whose blood volume
# pulses with the heart, as in the paper's in vivo experiment (Experiments,
# Fig. 2).  THb is modulated in time by a cardiac term plus a slower
# respiratory term; roaming specular highlights add high-frequency noise; the
# right view is shifted and its red channel slightly miscalibrated (a constant
# offset between the views).

@dataclasses.dataclass(frozen=True)
class PulseSpec:
    n_frames: int = 300
    fps: float = 30.0
    pulse_hz: float = 1.25
    pulse_depth: float = 0.03       # relative THb modulation
    resp_hz: float = 0.25
    resp_depth: float = 0.02
    n_highlights: int = 3           # specular spots per frame
    highlight_peak: float = 0.6     # blend towards white at a spot's centre
    shift_px: float = 8.0           # right view
    red_gain_right: float = 0.98    # right-view calibration mismatch


def pulse_thb_factor(spec: PulseSpec, frame: int, phase: float = 0.4) -> float:
    t = frame / spec.fps
    return (1.0 + spec.pulse_depth * math.sin(2 * math.pi * spec.pulse_hz * t + phase)
            + spec.resp_depth * math.sin(2 * math.pi * spec.resp_hz * t))


def pulse_video(height: int, width: int, spec: PulseSpec = PulseSpec(), config: int = 6,
                dtype: str = "f32", frames: Optional[Sequence[int]] = None
                ) -> Tuple[np.ndarray, np.ndarray]:
    """Stereo video [2][T][H][W][3] (storage dtype) and the true THb [2][T][H][W]."""
    sp = spectra()
    ft = make_blob_field(height, width, _seed(config, 0, 1))
    fs = make_blob_field(height, width, _seed(config, 0, 2))
    idx = list(range(spec.n_frames)) if frames is None else list(frames)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    out = np.empty((2, len(idx), height, width, 3), dtype=np.uint16 if dtype == "bf16" else
                   (np.float16 if dtype == "f16" else np.float32))
    thb_out = np.empty((2, len(idx), height, width))
    for view in range(2):
        thb0, so2 = truth(height, width, ft, fs, shift_x=view * spec.shift_px)
        for i, f in enumerate(idx):
            thb = thb0 * pulse_thb_factor(spec, f)
            hb, hbo2 = hb_hbo2(thb, so2)
            clean = render_intensity(hb, hbo2, sp)
            rng = np.random.default_rng(_seed(config, view, 5) * 100003 + f)
            spot = np.zeros((height, width))
            for _ in range(spec.n_highlights):
                cy, cx = rng.uniform(0, height), rng.uniform(0, width)
                sd = rng.uniform(0.01, 0.04) * min(height, width)
                spot = np.maximum(spot, spec.highlight_peak * rng.uniform(0.5, 1.0) *
                                  np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * sd * sd)))
            clean = clean + (1.0 - clean) * spot[..., None]
            if view == 1:
                clean[..., 0] *= spec.red_gain_right
            noisy = clean + rng.normal(0.0, NOISE_SIGMA, clean.shape)
            out[view, i] = quantise(noisy, dtype)
            thb_out[view, i] = thb
    return out, thb_out


# Serving workload: 16 streams of mixed resolution at 30 fps with Poisson arrivals.
SERVE_CLASSES = (  # (count, height, width, levels, grid)
    (4, 480, 640, 2, 256),
    (6, 1024, 1280, 1, 128),
    (4, 1080, 1920, 2, 256),
    (2, 2160, 3840, 2, 128),
)


@dataclasses.dataclass(frozen=True)
class StreamSpec:
    stream: int
    height: int
    width: int
    levels: int
    grid: int
    fps: float


def serve_streams(classes=SERVE_CLASSES, fps: float = 30.0) -> List[StreamSpec]:
    out, s = [], 0
    for count, h, w, lv, g in classes:
        for _ in range(count):
            out.append(StreamSpec(s, h, w, lv, g, fps))
            s += 1
    return out


def poisson_arrivals(stream: int, rate_hz: float, duration_s: float, config: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate, seeded per stream."""
    rng = np.random.default_rng(_seed(config, stream, 5))
    n = int(rate_hz * duration_s * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    return t[t < duration_s]
