"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers are built here with the sanitizers and run:
  * tests/c/oracle_asan.c with the FP64 oracle (gcc): every oracle function on
    ragged shapes, levels 0..3, both low-pass modes and the illumination term;
  * tests/c/plan_tables_asan.cpp with the library's host plan source (the
    host pass of hipcc only, no device code is instrumented): the FP64
    super-tile table and bf16 split-operand builders on ragged and square
    grids, and the host-side validation.
Leak checking is on; any report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fopenmp", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "c", "oracle_asan.c"), os.path.join(ROOT, "oracle", "hb_oracle.c"),
                    "-o", exe, "-lm"], check=True)
    assert "oracle asan ok" in _run(exe)


def test_plan_host_tables_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    clangxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not (os.path.exists(hipcc) and os.path.exists(clangxx)):
        pytest.skip("ROCm compilers not found")
    obj, exe = str(tmp_path / "pt.o"), str(tmp_path / "plan_tables_asan")
    # host pass only; each sanitizer flag goes to the host compiler
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only", "-std=c++17", "-O1", "-g",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1706_07263_amd", "csrc"),
                    "-c", os.path.join(ROOT, "tests", "c", "plan_tables_asan.cpp"), "-o", obj],
                   check=True, capture_output=True)
    # link (no HIP source on this line): the sanitizer runtimes and the HIP runtime
    subprocess.run([clangxx, "-fsanitize=address,undefined", obj, "-o", exe, "-L", os.path.join(ROCM, "lib"),
                    "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")], check=True)
    assert "plan tables asan ok" in _run(exe)
