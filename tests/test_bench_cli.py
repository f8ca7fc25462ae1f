"""bench.py's command line: defaults of the measured workload and the
one-GPU refusal (host logic only)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_defaults_are_the_video_workload(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.gpus, a.batch, a.dtype, a.levels, a.grid, a.split) == (1, 16, "f32", 2, 256, 0)
    assert a.steps >= 20 and a.warmup >= 1 and a.sequence == 0


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert r.stdout == ""
    assert "measures one GPU" in r.stderr


def test_kernel_source_hash_covers_the_device_sources():
    assert set(bench.KERNEL_SOURCES) >= {"hb_kernels.hip", "hb_internal.h", "hb_df.h"}
    h = bench.kernel_source_sha()
    assert len(h) == 16 and int(h, 16) >= 0
