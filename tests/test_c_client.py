"""The C ABI from a C program with no Python or PyTorch in the process
(tests/c/hb_client.c, built by __graft_entry__.build())."""
import os
import subprocess

import numpy as np
import pytest

from paper_1706_07263_amd import synth
from tests import hbtest

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "hb_client")


@pytest.fixture(scope="module")
def client():
    if not os.path.exists(EXE):
        from tests.c import build_client
        build_client.build()
    return EXE


def test_client_host_checks(client):
    out = subprocess.run([client, "check"], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert "host checks passed" in out.stdout


@pytest.mark.gpu
def test_client_estimates_match_oracle(client, tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sp = synth.spectra()
    h, w, levels, grid = 64, 96, 2, 48
    frames = np.stack([synth.single_frame(h, w, config=88, frame=f)[0] for f in range(3)]).astype(np.float32)
    fin = tmp_path / "frames.bin"
    frames.tofile(fin)
    with open(str(fin) + ".model", "wb") as f:
        f.write(np.int32(sp.eps_hb.size).tobytes() + b"\0" * 4)
        for a in (sp.eps_hb, sp.eps_hbo2, sp.response.reshape(-1), np.array([sp.path_length_cm])):
            f.write(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    fout = tmp_path / "maps.bin"
    out = subprocess.run([client, "run", str(fin), str(fout), str(w), str(h), str(levels), str(grid)],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    maps = np.fromfile(fout, dtype=np.float32).reshape(3, 4, h, w)
    s = synth.plan_settings(levels=levels, grid=grid)
    err = hbtest.assert_maps_close(maps, hbtest.run_oracle(frames, "f32", s), "C client")
    print("C client errors", err)
