"""Issue ceilings of the posterior kernel's instruction mix on the GPU
(ctypes binding of ``libhbceiling.so``, built from csrc/hb_ceiling.hip).

Measurement code for the benchmark's roofline, not part of the estimation
path.  Each microbenchmark is a register-only loop launched at a fixed number
of waves per SIMD on every compute unit; the result is a rate (work units per
second) from HIP events, and the SIMD cycles per wave instruction it implies
at the nominal clock.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhbceiling.so")

# MI355X: 256 compute units of 4 SIMDs, 2.4 GHz peak engine clock.
N_CU = 256
SIMD_PER_CU = 4
CLOCK_HZ = 2.4e9
WAVE = 64
PAIRS_PER_CHUNK_BLOCK = 256          # 16 nodes x 16 pixels per MFMA
VALU_PER_CHUNK_BLOCK = 9             # the posterior's chunk body besides MFMA and exp
EXP_PER_CHUNK_BLOCK = 4

KINDS = {"mix": 0, "fma": 1, "exp": 2, "mfma": 3, "mfma_fma": 4, "exp_fma": 5}
# loop iterations per wave sized for a few milliseconds per launch
ITERS = {"mix": 20000, "fma": 50000, "exp": 25000, "mfma": 50000, "mfma_fma": 40000, "exp_fma": 30000}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        L.hb_ceiling_measure.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.hb_ceiling_measure.restype = ctypes.c_int
        _lib = L
    return _lib


def measure(kind: str, waves_per_simd: int = 6, iters: int = 0, reps: int = 5) -> Dict[str, float]:
    """Rate of one microbenchmark: units/s and, for single-instruction kinds,
    SIMD cycles per wave instruction at CLOCK_HZ."""
    blocks = N_CU * SIMD_PER_CU * waves_per_simd // 4
    ms, units = ctypes.c_double(), ctypes.c_double()
    rc = lib().hb_ceiling_measure(KINDS[kind], blocks, iters or ITERS[kind], reps, ctypes.byref(ms),
                                  ctypes.byref(units))
    if rc != 0:
        raise RuntimeError(f"hb_ceiling_measure({kind}) failed: {rc}")
    rate = units.value / (ms.value * 1e-3)
    out = {"ms": ms.value, "units": units.value, "units_per_s": rate}
    simd_cycles_per_s = N_CU * SIMD_PER_CU * CLOCK_HZ
    if kind in ("fma", "exp", "exp_fma"):
        out["cycles_per_wave_instr"] = simd_cycles_per_s / (rate / WAVE)
    elif kind in ("mfma", "mfma_fma"):
        out["cycles_per_wave_instr"] = simd_cycles_per_s / rate
    elif kind == "mix":
        out["cycles_per_chunk_block"] = simd_cycles_per_s / (rate / PAIRS_PER_CHUNK_BLOCK)
    return out


def ceilings(waves_per_simd: int = 6) -> Dict[str, object]:
    """All microbenchmarks, the measured ceiling of the posterior's chunk mix
    (pairs/s) and the ceiling predicted from the separate instruction costs
    if the matrix, transcendental and FMA work did not overlap."""
    r = {k: measure(k, waves_per_simd) for k in KINDS}
    c_fma = r["fma"]["cycles_per_wave_instr"]
    c_exp = r["exp"]["cycles_per_wave_instr"]
    c_mfma = r["mfma"]["cycles_per_wave_instr"]
    serial = c_mfma + EXP_PER_CHUNK_BLOCK * c_exp + VALU_PER_CHUNK_BLOCK * c_fma
    simd_cycles_per_s = N_CU * SIMD_PER_CU * CLOCK_HZ
    return {
        "waves_per_simd": waves_per_simd,
        "clock_hz_assumed": CLOCK_HZ,
        "mix_pairs_per_s": r["mix"]["units_per_s"],
        "mix_cycles_per_chunk_block": r["mix"]["cycles_per_chunk_block"],
        "fma_lane_ops_per_s": r["fma"]["units_per_s"],
        "exp_lane_ops_per_s": r["exp"]["units_per_s"],
        "mfma_16x16x32_bf16_per_s": r["mfma"]["units_per_s"],
        "cycles_per_wave_instr": {"fma": c_fma, "exp": c_exp, "mfma_16x16x32_bf16": c_mfma},
        "mfma_with_16_fma_cycles": r["mfma_fma"]["cycles_per_wave_instr"],
        "mfma_plus_16_fma_if_serial_cycles": c_mfma + 16 * c_fma,
        "exp_with_fma_cycles_per_pair": simd_cycles_per_s / (r["exp_fma"]["units_per_s"] / WAVE),
        "exp_plus_fma_if_serial_cycles": c_exp + c_fma,
        "chunk_block_cycles_if_serial": serial,
        "serial_model_pairs_per_s": PAIRS_PER_CHUNK_BLOCK * simd_cycles_per_s / serial,
    }


if __name__ == "__main__":
    import json
    print(json.dumps(ceilings(), indent=1))
