"""ctypes wrapper of the FP64 CPU oracle (hb_oracle.c).

TEST INFRASTRUCTURE ONLY: the reference the GPU path is checked against.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg import it.
It shares no code with the GPU library.

The library is compiled with plain gcc (-O2, no fast-math, OpenMP) into
``oracle/libhb_oracle.so``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhb_oracle.so")
SRC_PATH = os.path.join(HERE, "hb_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc.  Returns the library path."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               SRC_PATH, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_mu.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, dp]
        L.orc_jacobian.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, dp]
        L.orc_tikhonov.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp, dp]
        L.orc_tikhonov.restype = ctypes.c_int
        L.orc_grid.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, dp]
        L.orc_haar_forward.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_haar_inverse.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_posterior_mean.argtypes = [dp, dp, ctypes.c_long, dp, ctypes.c_double, ctypes.c_int, dp]
        L.orc_estimate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, dp, ctypes.c_int, dp]
        L.orc_estimate.restype = ctypes.c_int
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


class _Model(ctypes.Structure):
    _fields_ = [("n_wl", ctypes.c_int),
                ("eps_hb", ctypes.POINTER(ctypes.c_double)),
                ("eps_hbo2", ctypes.POINTER(ctypes.c_double)),
                ("response", ctypes.POINTER(ctypes.c_double)),
                ("path_cm", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("height", ctypes.c_int), ("levels", ctypes.c_int),
                ("grid_thb", ctypes.c_int), ("grid_so2", ctypes.c_int),
                ("thb_min", ctypes.c_double), ("thb_max", ctypes.c_double),
                ("so2_min", ctypes.c_double), ("so2_max", ctypes.c_double),
                ("lambda_rel", ctypes.c_double), ("sigma", ctypes.c_double),
                ("floor", ctypes.c_double), ("thb_eps", ctypes.c_double),
                ("ref_hb", ctypes.c_double), ("ref_hbo2", ctypes.c_double),
                ("lowpass", ctypes.c_int), ("illumination", ctypes.c_int)]


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclasses.dataclass
class Model:
    """Camera sensitivities and attenuation spectra."""
    eps_hb: np.ndarray
    eps_hbo2: np.ndarray
    response: np.ndarray     # [3][n]
    path_cm: float

    def __post_init__(self):
        self.eps_hb = np.ascontiguousarray(self.eps_hb, dtype=np.float64)
        self.eps_hbo2 = np.ascontiguousarray(self.eps_hbo2, dtype=np.float64)
        self.response = np.ascontiguousarray(self.response, dtype=np.float64)
        assert self.response.shape == (3, self.eps_hb.size)

    def c_struct(self) -> _Model:
        return _Model(self.eps_hb.size, _dp(self.eps_hb), _dp(self.eps_hbo2),
                      _dp(self.response), float(self.path_cm))


@dataclasses.dataclass
class Params:
    width: int
    height: int
    levels: int = 1
    grid_thb: int = 32
    grid_so2: int = 32
    thb_min: float = 20.0
    thb_max: float = 200.0
    so2_min: float = 0.3
    so2_max: float = 1.0
    lambda_rel: float = 1e-3
    sigma: float = 0.01
    floor: float = 1e-4
    thb_eps: float = 1e-3
    ref_hb: Optional[float] = None     # default: grid centre
    ref_hbo2: Optional[float] = None
    lowpass: int = 0                   # 0 Bayesian, 1 Tikhonov
    illumination: int = 0              # 1: integrate out a per-pixel log offset

    def ref(self) -> Tuple[float, float]:
        if self.ref_hb is not None and self.ref_hbo2 is not None:
            return float(self.ref_hb), float(self.ref_hbo2)
        thb = 0.5 * (self.thb_min + self.thb_max)
        so2 = 0.5 * (self.so2_min + self.so2_max)
        return thb * (1.0 - so2), thb * so2

    def c_struct(self) -> _Params:
        rh, ro = self.ref()
        return _Params(self.width, self.height, self.levels, self.grid_thb, self.grid_so2,
                       self.thb_min, self.thb_max, self.so2_min, self.so2_max,
                       self.lambda_rel, self.sigma, self.floor, self.thb_eps, rh, ro,
                       self.lowpass, self.illumination)


def mu(model: Model, hb: float, hbo2: float) -> np.ndarray:
    out = np.zeros(3)
    m = model.c_struct()
    lib().orc_mu(ctypes.byref(m), hb, hbo2, _dp(out))
    return out


def jacobian(model: Model, hb: float, hbo2: float) -> np.ndarray:
    out = np.zeros(6)
    m = model.c_struct()
    lib().orc_jacobian(ctypes.byref(m), hb, hbo2, _dp(out))
    return out.reshape(3, 2)


def tikhonov(E: np.ndarray, lambda_rel: float) -> Tuple[np.ndarray, float]:
    E = np.ascontiguousarray(E, dtype=np.float64)
    rows = E.shape[0]
    M = np.zeros(2 * rows)
    g = np.zeros(1)
    rc = lib().orc_tikhonov(rows, _dp(E), lambda_rel, _dp(M), _dp(g))
    if rc != 0:
        raise np.linalg.LinAlgError("singular Tikhonov system")
    return M.reshape(2, rows), float(g[0])


def grid(params: Params, model: Model) -> Tuple[np.ndarray, np.ndarray]:
    G = params.grid_thb * params.grid_so2
    c = np.zeros(G * 2)
    m_ = np.zeros(G * 3)
    p = params.c_struct()
    m = model.c_struct()
    lib().orc_grid(ctypes.byref(p), ctypes.byref(m), _dp(c), _dp(m_))
    return c.reshape(G, 2), m_.reshape(G, 3)


def haar_forward(x: np.ndarray, levels: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    lib().orc_haar_forward(_dp(x), x.shape[0], x.shape[1], levels, _dp(out))
    return out


def haar_inverse(c: np.ndarray, levels: int) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros_like(c)
    lib().orc_haar_inverse(_dp(c), c.shape[0], c.shape[1], levels, _dp(out))
    return out


def posterior_mean(c: np.ndarray, mu_: np.ndarray, ybar, sigma: float, illumination: int = 0) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.float64)
    mu_ = np.ascontiguousarray(mu_, dtype=np.float64)
    y = np.ascontiguousarray(ybar, dtype=np.float64)
    out = np.zeros(2)
    lib().orc_posterior_mean(_dp(c), _dp(mu_), c.shape[0], _dp(y), sigma, int(illumination), _dp(out))
    return out


def estimate(params: Params, model: Model, frames: np.ndarray) -> np.ndarray:
    """frames [N][H][W][3] (any float dtype, widened exactly to float64) ->
    maps [N][4][H][W] float64 (Hb, HbO2, THb, SO2)."""
    fr = np.ascontiguousarray(frames, dtype=np.float64)
    if fr.ndim == 3:
        fr = fr[None]
    n, h, w, ch = fr.shape
    assert ch == 3 and h == params.height and w == params.width
    out = np.zeros((n, 4, h, w))
    p = params.c_struct()
    m = model.c_struct()
    rc = lib().orc_estimate(ctypes.byref(p), ctypes.byref(m), _dp(fr), n, _dp(out))
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (code {rc})")
    return out


def threads() -> int:
    return int(lib().orc_threads())
