"""Pins of the oracle's forward model and its linearisation."""
import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import hb_oracle as orc


def test_zero_concentration_has_zero_attenuation(model):
    assert np.max(np.abs(orc.mu(model, 0.0, 0.0))) < 1e-15


def test_single_wavelength_response_is_beer_lambert(spectra):
    """A camera channel that sees one wavelength reduces to Beer-Lambert:
    mu = L (eps_hb c_hb + eps_hbo2 c_hbo2)."""
    n = spectra.eps_hb.size
    picks = [10, 28, 45]
    resp = np.zeros((3, n))
    for k, j in enumerate(picks):
        resp[k, j] = 0.7   # any positive scale: responses are normalised
    m = orc.Model(spectra.eps_hb, spectra.eps_hbo2, resp, 0.1)
    for hb, hbo2 in [(0.0, 0.0), (40.0, 80.0), (130.0, 5.0)]:
        got = orc.mu(m, hb, hbo2)
        want = np.array([0.1 * (spectra.eps_hb[j] * hb + spectra.eps_hbo2[j] * hbo2) for j in picks])
        assert np.allclose(got, want, rtol=1e-14, atol=1e-15)


def test_mu_is_increasing_in_concentration(model):
    base = orc.mu(model, 50.0, 50.0)
    assert np.all(orc.mu(model, 60.0, 50.0) > base)
    assert np.all(orc.mu(model, 50.0, 60.0) > base)


@pytest.mark.parametrize("c", [(0.0, 0.0), (38.5, 71.5), (100.0, 20.0), (5.0, 190.0)])
def test_jacobian_matches_complex_step(model, spectra, c):
    E = orc.jacobian(model, *c)
    Ecs = bf.jacobian_complex_step(c, spectra.eps_hb, spectra.eps_hbo2, spectra.response,
                                   spectra.path_length_cm)
    assert np.allclose(E, Ecs, rtol=1e-12, atol=0)


def test_grid_is_inclusive_product_grid(model):
    p = orc.Params(width=2, height=2, grid_thb=5, grid_so2=3, thb_min=20, thb_max=200,
                   so2_min=0.3, so2_max=1.0)
    c, mu = orc.grid(p, model)
    thb = c.sum(axis=1).reshape(5, 3)
    so2 = (c[:, 1] / c.sum(axis=1)).reshape(5, 3)
    assert np.allclose(thb[:, 0], [20, 65, 110, 155, 200])
    assert np.allclose(so2[0], [0.3, 0.65, 1.0])
    for g in (0, 7, 14):
        assert np.allclose(mu[g], orc.mu(model, *c[g]), rtol=0, atol=0)
