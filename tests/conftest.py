import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name: str) -> np.ndarray:
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


@pytest.fixture(scope="session")
def spectra():
    from paper_1706_07263_amd import synth
    return synth.spectra()


@pytest.fixture(scope="session")
def model(spectra):
    from oracle import hb_oracle as orc
    return orc.Model(spectra.eps_hb, spectra.eps_hbo2, spectra.response, spectra.path_length_cm)
