"""Thin ctypes binding of the C ABI in include/hb.h (argument marshalling only).

Every step of the estimation runs in the HIP library ``libhbgpu.so`` built
in-tree next to this file; if it is missing, importing this module fails.
There is no CPU fallback.

Functions keep the C names (``hb_plan_create`` ...).  ``Plan`` wraps them for
PyTorch callers: frames and maps are CUDA (HIP) tensors, the stream is the
current torch stream unless one is given.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhbgpu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(or python paper_1706_07263_amd/build.py) first")

_lib = ctypes.CDLL(LIB_PATH)

HB_OK = 0
HB_ERR_INVALID_ARG = -1
HB_ERR_SHAPE = -2
HB_ERR_NO_FORWARD_MODEL = -3
HB_ERR_OUT_OF_MEMORY = -4
HB_ERR_DEVICE = -5
HB_ERR_ILL_POSED = -6
HB_ERR_BATCH = -7
HB_ERR_SCRATCH = -8
HB_NOALLOC_SCRATCH_BYTES = 128 << 20

HB_F32, HB_F16, HB_BF16 = 0, 1, 2
HB_LOWPASS_BAYES, HB_LOWPASS_TIKHONOV = 0, 1
HB_DEBUG_LOWPASS_OBS, HB_DEBUG_DETAILS, HB_DEBUG_LOWPASS_EST = 0, 1, 2
HB_DEBUG_NODE_OPERANDS, HB_DEBUG_SPLIT_OPERANDS = 3, 4

DTYPES = {"f32": HB_F32, "f16": HB_F16, "bf16": HB_BF16}


class hb_plan_desc_t(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("frame_dtype", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("grid_thb", ctypes.c_int32), ("grid_so2", ctypes.c_int32),
                ("thb_min", ctypes.c_double), ("thb_max", ctypes.c_double),
                ("so2_min", ctypes.c_double), ("so2_max", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("sigma", ctypes.c_double),
                ("intensity_floor", ctypes.c_double),
                ("ref_thb", ctypes.c_double), ("ref_so2", ctypes.c_double),
                ("thb_eps", ctypes.c_double),
                ("lowpass", ctypes.c_int32), ("grid_split", ctypes.c_int32),
                ("illumination", ctypes.c_int32), ("posterior_tolerance", ctypes.c_double)]


class hb_forward_model_t(ctypes.Structure):
    _fields_ = [("n_wavelengths", ctypes.c_int32),
                ("wavelength_nm", ctypes.POINTER(ctypes.c_double)),
                ("eps_hb", ctypes.POINTER(ctypes.c_double)),
                ("eps_hbo2", ctypes.POINTER(ctypes.c_double)),
                ("response", ctypes.POINTER(ctypes.c_double)),
                ("path_length_cm", ctypes.c_double)]


class hb_maps_t(ctypes.Structure):
    _fields_ = [("hb", ctypes.c_void_p), ("hbo2", ctypes.c_void_p),
                ("thb", ctypes.c_void_p), ("so2", ctypes.c_void_p)]


class hb_plan_info_t(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double * 6), ("M", ctypes.c_double * 6), ("gamma", ctypes.c_double),
                ("ref_hb", ctypes.c_double), ("ref_hbo2", ctypes.c_double),
                ("mu_ref", ctypes.c_double * 3), ("grid_split", ctypes.c_int32),
                ("n_tiles", ctypes.c_int32), ("posterior_kernel", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64), ("skip_log2", ctypes.c_double), ("skip_bound", ctypes.c_double),
                ("mfma_index", ctypes.c_double), ("direct_index", ctypes.c_double),
                ("band_log2", ctypes.c_double), ("band_chunks", ctypes.c_int64),
                ("far_room", ctypes.c_double), ("mfma_df_constant", ctypes.c_int32),
                ("m_norm", ctypes.c_double),
                ("k1_double_float", ctypes.c_int32)]


_P = ctypes.c_void_p
_lib.hb_plan_desc_default.argtypes = [ctypes.POINTER(hb_plan_desc_t)]
_lib.hb_plan_create.argtypes = [ctypes.POINTER(hb_plan_desc_t), ctypes.c_int, ctypes.POINTER(_P)]
_lib.hb_set_forward_model.argtypes = [_P, ctypes.POINTER(hb_forward_model_t)]
_lib.hb_estimate_frames.argtypes = [_P, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(hb_maps_t),
                                    ctypes.c_void_p]
_lib.hb_estimate_frames_noalloc.argtypes = [_P, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(hb_maps_t),
                                            ctypes.c_void_p]
_lib.hb_destroy.argtypes = [_P]
_lib.hb_status_string.argtypes = [ctypes.c_int]
_lib.hb_status_string.restype = ctypes.c_char_p
_lib.hb_plan_device_bytes.argtypes = [_P]
_lib.hb_plan_device_bytes.restype = ctypes.c_size_t
_lib.hb_plan_get_info.argtypes = [_P, ctypes.POINTER(hb_plan_info_t)]
_lib.hb_plan_set_timing.argtypes = [_P, ctypes.c_int32]
_lib.hb_plan_get_timing.argtypes = [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
_lib.hb_debug_copy.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]
_lib.hb_plan_get_work.argtypes = [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
_lib.hb_plan_get_far_pixels.argtypes = [_P, ctypes.POINTER(ctypes.c_int64)]
for _f in ("hb_plan_desc_default", "hb_plan_create", "hb_set_forward_model", "hb_estimate_frames",
           "hb_estimate_frames_noalloc", "hb_destroy", "hb_plan_get_info", "hb_plan_set_timing", "hb_plan_get_timing", "hb_debug_copy",
           "hb_plan_get_work", "hb_plan_get_far_pixels"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("hb_plan_desc_default", "hb_plan_create", "hb_set_forward_model", "hb_estimate_frames",
            "hb_estimate_frames_noalloc", "hb_destroy", "hb_status_string", "hb_plan_device_bytes", "hb_plan_get_info",
            "hb_plan_set_timing", "hb_plan_get_timing", "hb_debug_copy", "hb_plan_get_work",
            "hb_plan_get_far_pixels")


class HbError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {hb_status_string(status)} ({status})")
        self.status = status


def _check(status: int, where: str) -> None:
    if status != HB_OK:
        raise HbError(status, where)


# --- C-named functions -------------------------------------------------------

def hb_status_string(status: int) -> str:
    return _lib.hb_status_string(status).decode()


def hb_plan_desc_default() -> hb_plan_desc_t:
    d = hb_plan_desc_t()
    _check(_lib.hb_plan_desc_default(ctypes.byref(d)), "hb_plan_desc_default")
    return d


def hb_plan_create(desc: hb_plan_desc_t, device: int = 0) -> int:
    h = _P()
    _check(_lib.hb_plan_create(ctypes.byref(desc), device, ctypes.byref(h)), "hb_plan_create")
    return h.value


def hb_set_forward_model(plan: int, eps_hb, eps_hbo2, response, path_length_cm: float,
                         wavelength_nm=None) -> None:
    ehb = np.ascontiguousarray(eps_hb, dtype=np.float64)
    eox = np.ascontiguousarray(eps_hbo2, dtype=np.float64)
    resp = np.ascontiguousarray(response, dtype=np.float64)
    if resp.shape != (3, ehb.size) or eox.size != ehb.size:
        raise ValueError("response must be [3][n] and eps arrays [n]")
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    wl = None if wavelength_nm is None else np.ascontiguousarray(wavelength_nm, dtype=np.float64)
    fm = hb_forward_model_t(ehb.size, dp(wl) if wl is not None else None, dp(ehb), dp(eox), dp(resp),
                            float(path_length_cm))
    _check(_lib.hb_set_forward_model(_P(plan), ctypes.byref(fm)), "hb_set_forward_model")


def hb_estimate_frames(plan: int, d_frames: int, n_frames: int, maps: Sequence[int],
                       stream: int = 0) -> None:
    m = hb_maps_t(*[int(x) if x else None for x in maps])
    _check(_lib.hb_estimate_frames(_P(plan), ctypes.c_void_p(d_frames), n_frames, ctypes.byref(m),
                                   ctypes.c_void_p(stream)), "hb_estimate_frames")


def hb_estimate_frames_noalloc(plan: int, d_frames: int, n_frames: int, maps: Sequence[int],
                               stream: int = 0) -> None:
    m = hb_maps_t(*[int(x) if x else None for x in maps])
    _check(_lib.hb_estimate_frames_noalloc(_P(plan), ctypes.c_void_p(d_frames), n_frames, ctypes.byref(m),
                                           ctypes.c_void_p(stream)), "hb_estimate_frames_noalloc")


def hb_destroy(plan: int) -> None:
    _check(_lib.hb_destroy(_P(plan)), "hb_destroy")


def hb_plan_device_bytes(plan: int) -> int:
    return int(_lib.hb_plan_device_bytes(_P(plan)))


def hb_plan_get_info(plan: int) -> Dict[str, object]:
    info = hb_plan_info_t()
    _check(_lib.hb_plan_get_info(_P(plan), ctypes.byref(info)), "hb_plan_get_info")
    return dict(E=np.array(info.E[:]).reshape(3, 2), M=np.array(info.M[:]).reshape(2, 3),
                gamma=info.gamma, ref=(info.ref_hb, info.ref_hbo2), mu_ref=np.array(info.mu_ref[:]),
                grid_split=info.grid_split, n_tiles=info.n_tiles, n_nodes=info.n_nodes,
                posterior_kernel=("mfma", "direct", "direct_precise")[info.posterior_kernel],
                skip_log2=info.skip_log2, skip_bound=info.skip_bound, mfma_index=info.mfma_index,
                direct_index=info.direct_index, band_log2=info.band_log2, band_chunks=info.band_chunks,
                far_room=info.far_room, mfma_df_constant=bool(info.mfma_df_constant),
                m_norm=info.m_norm,
                k1_double_float=bool(info.k1_double_float))


def hb_plan_set_timing(plan: int, enable: bool) -> None:
    _check(_lib.hb_plan_set_timing(_P(plan), int(bool(enable))), "hb_plan_set_timing")


def hb_plan_get_timing(plan: int) -> Tuple[np.ndarray, np.ndarray]:
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    _check(_lib.hb_plan_get_timing(_P(plan), ms, n), "hb_plan_get_timing")
    return np.array(ms[:]), np.array(n[:])


def hb_plan_get_work(plan: int) -> Tuple[int, int]:
    ev = ctypes.c_int64()
    full = ctypes.c_int64()
    _check(_lib.hb_plan_get_work(_P(plan), ctypes.byref(ev), ctypes.byref(full)), "hb_plan_get_work")
    return ev.value, full.value


def hb_plan_get_far_pixels(plan: int) -> int:
    n = ctypes.c_int64()
    _check(_lib.hb_plan_get_far_pixels(_P(plan), ctypes.byref(n)), "hb_plan_get_far_pixels")
    return n.value


def hb_debug_copy(plan: int, which: int, frame: int, out: np.ndarray) -> np.ndarray:
    assert out.flags.c_contiguous
    _check(_lib.hb_debug_copy(_P(plan), which, frame, out.ctypes.data, out.nbytes), "hb_debug_copy")
    return out


# --- PyTorch-facing wrapper --------------------------------------------------

def make_desc(width: int, height: int, levels: int = 1, dtype: str = "f32", max_batch: int = 1,
              grid_thb: int = 128, grid_so2: int = 128, thb_min: float = 20.0, thb_max: float = 200.0,
              so2_min: float = 0.3, so2_max: float = 1.0, lam: float = 1e-3, sigma: float = 0.01,
              intensity_floor: float = 1e-4, ref_thb: float = math.nan, ref_so2: float = math.nan,
              thb_eps: float = 1e-3, lowpass: int = HB_LOWPASS_BAYES, grid_split: int = 0,
              illumination: int = 0, posterior_tolerance: Optional[float] = None) -> hb_plan_desc_t:
    d = hb_plan_desc_default()
    d.width, d.height, d.levels = width, height, levels
    d.frame_dtype = DTYPES[dtype]
    d.max_batch = max_batch
    d.grid_thb, d.grid_so2 = grid_thb, grid_so2
    d.thb_min, d.thb_max, d.so2_min, d.so2_max = thb_min, thb_max, so2_min, so2_max
    d.lambda_, d.sigma, d.intensity_floor = lam, sigma, intensity_floor
    d.ref_thb, d.ref_so2, d.thb_eps = ref_thb, ref_so2, thb_eps
    d.lowpass, d.grid_split = lowpass, grid_split
    d.illumination = illumination
    if posterior_tolerance is not None:
        d.posterior_tolerance = posterior_tolerance
    return d


class Plan:
    """Owns one hb_plan_t.  Use as a context manager or call close()."""

    def __init__(self, desc: hb_plan_desc_t, device: int = 0):
        self.desc = desc
        self.device = device
        self.handle = hb_plan_create(desc, device)

    def set_forward_model(self, spectra) -> "Plan":
        hb_set_forward_model(self.handle, spectra.eps_hb, spectra.eps_hbo2, spectra.response,
                             spectra.path_length_cm, getattr(spectra, "wavelength_nm", None))
        return self

    def estimate(self, frames, maps: Sequence, stream=None, noalloc: bool = False) -> None:
        """frames: device tensor [n][H][W][3] (float32/float16, or int16/uint16
        bit patterns for bfloat16); maps: four device float32 tensors
        [n][H][W] or None.  Shapes, dtypes, devices and contiguity are checked
        here, since the library receives bare pointers.  noalloc: call
        hb_estimate_frames_noalloc (intermediate buffers in the library's
        static scratch) instead of hb_estimate_frames."""
        import torch
        d = self.desc
        want = {HB_F32: (torch.float32,), HB_F16: (torch.float16,),
                HB_BF16: (torch.int16, torch.uint16, torch.bfloat16)}[d.frame_dtype]
        if frames.dtype not in want:
            raise HbError(HB_ERR_INVALID_ARG, f"frames dtype {frames.dtype}, plan expects {want}")
        if frames.dim() != 4 or tuple(frames.shape[1:]) != (d.height, d.width, 3):
            raise HbError(HB_ERR_SHAPE, f"frames shape {tuple(frames.shape)}, plan expects "
                                        f"[n][{d.height}][{d.width}][3]")
        if not frames.is_cuda or not frames.is_contiguous():
            raise HbError(HB_ERR_INVALID_ARG, "frames must be a contiguous device tensor")
        n = frames.shape[0]
        if len(maps) != 4:
            raise HbError(HB_ERR_INVALID_ARG, "maps: four tensors or None (Hb, HbO2, THb, SO2)")
        for m in maps:
            if m is None:
                continue
            if (m.dtype != torch.float32 or not m.is_cuda or not m.is_contiguous()
                    or m.numel() < n * d.height * d.width or m.device != frames.device):
                raise HbError(HB_ERR_INVALID_ARG, "each map must be a contiguous float32 tensor on the frames' "
                                                  f"device with at least {n}x{d.height}x{d.width} values")
        ptrs = [m.data_ptr() if m is not None else 0 for m in maps]
        if stream is None:
            stream = torch.cuda.current_stream(frames.device)
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        call = hb_estimate_frames_noalloc if noalloc else hb_estimate_frames
        call(self.handle, frames.data_ptr(), n, ptrs, sp)

    def info(self) -> Dict[str, object]:
        return hb_plan_get_info(self.handle)

    def device_bytes(self) -> int:
        return hb_plan_device_bytes(self.handle)

    def close(self) -> None:
        if self.handle:
            hb_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
