"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, the ctypes structs match the C layout, and host-side argument
validation rejects bad plans before touching the device."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hb.h")


@pytest.fixture(scope="module")
def hb():
    lib = os.path.join(ROOT, "paper_1706_07263_amd", "libhbgpu.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    from paper_1706_07263_amd import hb as mod
    return mod


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hb_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(hb):
    names = declared_functions()
    assert len(names) >= 11
    lib = ctypes.CDLL(hb.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(hb.EXPORTED)


def test_struct_layout_matches_header(hb, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "hb.h"
#define F(T, m) printf(#T "." #m " %zu\\n", offsetof(T, m));
int main(void) {
  printf("hb_plan_desc_t %zu\\n", sizeof(hb_plan_desc_t));
  printf("hb_forward_model_t %zu\\n", sizeof(hb_forward_model_t));
  printf("hb_maps_t %zu\\n", sizeof(hb_maps_t));
  printf("hb_plan_info_t %zu\\n", sizeof(hb_plan_info_t));
  F(hb_plan_desc_t, thb_min) F(hb_plan_desc_t, lambda) F(hb_plan_desc_t, ref_thb)
  F(hb_plan_desc_t, lowpass) F(hb_plan_desc_t, grid_split) F(hb_plan_desc_t, illumination) F(hb_plan_desc_t, posterior_tolerance)
  F(hb_forward_model_t, eps_hb) F(hb_forward_model_t, path_length_cm)
  F(hb_plan_info_t, gamma) F(hb_plan_info_t, grid_split) F(hb_plan_info_t, posterior_kernel) F(hb_plan_info_t, n_nodes) F(hb_plan_info_t, skip_log2) F(hb_plan_info_t, skip_bound) F(hb_plan_info_t, mfma_index) F(hb_plan_info_t, direct_index) F(hb_plan_info_t, band_log2) F(hb_plan_info_t, band_chunks) F(hb_plan_info_t, far_room) F(hb_plan_info_t, mfma_df_constant) F(hb_plan_info_t, m_norm) F(hb_plan_info_t, k1_double_float)
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.splitlines())
    assert int(out["hb_plan_desc_t"]) == ctypes.sizeof(hb.hb_plan_desc_t)
    assert int(out["hb_forward_model_t"]) == ctypes.sizeof(hb.hb_forward_model_t)
    assert int(out["hb_maps_t"]) == ctypes.sizeof(hb.hb_maps_t)
    assert int(out["hb_plan_info_t"]) == ctypes.sizeof(hb.hb_plan_info_t)
    py = {"lambda": "lambda_"}
    for key, off in out.items():
        if "." in key:
            t, m = key.split(".")
            assert getattr(getattr(hb, t), py.get(m, m)).offset == int(off), key


def test_status_strings(hb):
    for s in range(0, -9, -1):
        assert hb.hb_status_string(s) and hb.hb_status_string(s) != "unknown status"
    assert hb.hb_status_string(-99) == "unknown status"


def test_defaults(hb):
    d = hb.hb_plan_desc_default()
    assert (d.width, d.height, d.levels, d.max_batch) == (64, 64, 1, 1)
    assert d.illumination == 0 and d.posterior_tolerance == 1e-6
    assert (d.grid_thb, d.grid_so2) == (128, 128)
    assert d.lambda_ == 1e-3 and d.sigma == 0.01 and d.intensity_floor == 1e-4
    assert math.isnan(d.ref_thb) and math.isnan(d.ref_so2)


BAD = [
    (dict(width=63), "HB_ERR_SHAPE"),
    (dict(width=0), "HB_ERR_SHAPE"),
    (dict(height=60, levels=3), "HB_ERR_SHAPE"),
    (dict(levels=6), "HB_ERR_INVALID_ARG"),
    (dict(levels=-1), "HB_ERR_INVALID_ARG"),
    (dict(frame_dtype=7), "HB_ERR_INVALID_ARG"),
    (dict(max_batch=0), "HB_ERR_INVALID_ARG"),
    (dict(grid_thb=0), "HB_ERR_INVALID_ARG"),
    (dict(grid_so2=5000), "HB_ERR_INVALID_ARG"),
    (dict(thb_max=10.0), "HB_ERR_INVALID_ARG"),
    (dict(so2_max=1.5), "HB_ERR_INVALID_ARG"),
    (dict(lambda_=-1.0), "HB_ERR_INVALID_ARG"),
    (dict(sigma=0.0), "HB_ERR_INVALID_ARG"),
    (dict(sigma=math.inf), "HB_ERR_INVALID_ARG"),
    (dict(intensity_floor=0.0), "HB_ERR_INVALID_ARG"),
    (dict(ref_thb=50.0), "HB_ERR_INVALID_ARG"),          # one of the pair NaN
    (dict(ref_thb=50.0, ref_so2=1.5), "HB_ERR_INVALID_ARG"),
    (dict(lowpass=2), "HB_ERR_INVALID_ARG"),
    (dict(grid_split=-1), "HB_ERR_INVALID_ARG"),
    (dict(illumination=2), "HB_ERR_INVALID_ARG"),
    (dict(posterior_tolerance=-math.inf), "HB_ERR_INVALID_ARG"),   # negative finite = no skipping
    (dict(posterior_tolerance=float("nan")), "HB_ERR_INVALID_ARG"),
]


@pytest.mark.parametrize("change,status", BAD)
def test_plan_create_rejects_before_device(hb, change, status):
    d = hb.hb_plan_desc_default()
    for k, v in change.items():
        setattr(d, k, v)
    with pytest.raises(hb.HbError) as e:
        hb.hb_plan_create(d, 0)
    assert e.value.status == getattr(hb, status)


def test_null_arguments(hb):
    lib = hb._lib
    assert lib.hb_plan_create(None, 0, None) == hb.HB_ERR_INVALID_ARG
    assert lib.hb_plan_desc_default(None) == hb.HB_ERR_INVALID_ARG
    assert lib.hb_set_forward_model(None, None) == hb.HB_ERR_INVALID_ARG
    m = hb.hb_maps_t()
    assert lib.hb_estimate_frames(None, None, 1, ctypes.byref(m), None) == hb.HB_ERR_INVALID_ARG
    assert lib.hb_destroy(None) == hb.HB_OK
    assert lib.hb_plan_device_bytes(None) == 0
    assert lib.hb_plan_set_timing(None, 1) == hb.HB_ERR_INVALID_ARG
    assert lib.hb_plan_get_info(None, None) == hb.HB_ERR_INVALID_ARG
    assert lib.hb_debug_copy(None, 0, 0, None, 0) == hb.HB_ERR_INVALID_ARG
    assert lib.hb_plan_get_work(None, None, None) == hb.HB_ERR_INVALID_ARG
    assert lib.hb_plan_get_far_pixels(None, None) == hb.HB_ERR_INVALID_ARG


def test_library_has_no_cpu_fallback_symbols(hb):
    """The product path is the HIP library; nothing in it links the oracle."""
    out = subprocess.run(["nm", "-D", "--defined-only", hb.LIB_PATH], capture_output=True, text=True).stdout
    assert "orc_" not in out


def test_noalloc_scratch_size_matches_header(hb):
    m = re.search(r"#define HB_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == hb.HB_NOALLOC_SCRATCH_BYTES


def test_noalloc_rejects_null_plan_on_the_host(hb):
    maps = hb.hb_maps_t()
    for fn in (hb._lib.hb_estimate_frames, hb._lib.hb_estimate_frames_noalloc):
        assert fn(None, None, 1, ctypes.byref(maps), None) == hb.HB_ERR_INVALID_ARG
        assert fn(None, None, 1, None, None) == hb.HB_ERR_INVALID_ARG
