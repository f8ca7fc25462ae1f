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


def _transmittance(spectra, j, hb, hbo2, path_cm):
    """Beer-Lambert transmittance at one wavelength (natural-log extinction)."""
    return np.exp(-path_cm * (spectra.eps_hb[j] * hb + spectra.eps_hbo2[j] * hbo2))


@pytest.mark.parametrize("c", [(40.0, 80.0), (150.0, 10.0), (5.0, 3.0)])
def test_two_wavelength_channel_averages_transmittances(spectra, c):
    """Camera intensities are a linear map of the spectral intensities (Method,
    Eq. 3), and each wavelength attenuates by Beer-Lambert: a channel that sees
    two wavelengths with equal sensitivity receives the mean of their
    transmittances, exp(-mu) = (T1 + T2) / 2 (not their geometric mean, which
    mixing in the log domain would give)."""
    n = spectra.eps_hb.size
    j1, j2, j3 = 4, 50, 30          # 420 nm (strong absorption), 650 nm (weak), 550 nm
    resp = np.zeros((3, n))
    resp[0, [j1, j2]] = 2.5          # equal weights, any scale
    resp[1, [j1, j3]] = [1.0, 3.0]   # weights 1/4 and 3/4
    resp[2, [j2, j3]] = [0.2, 0.2]
    L = 0.1
    m = orc.Model(spectra.eps_hb, spectra.eps_hbo2, resp, L)
    hb, hbo2 = c
    t1, t2, t3 = (_transmittance(spectra, j, hb, hbo2, L) for j in (j1, j2, j3))
    got = np.exp(-orc.mu(m, hb, hbo2))
    want = np.array([(t1 + t2) / 2, 0.25 * t1 + 0.75 * t3, (t2 + t3) / 2])
    assert np.allclose(got, want, rtol=1e-14, atol=0)
    # the two transmittances differ enough for the distinction to matter
    assert abs(t1 - t2) > 1e-3


@pytest.mark.parametrize("alpha", [0.25, 0.6])
def test_channel_transmittance_is_linear_in_the_response(spectra, alpha):
    """Superposition (Method, Eq. 3: I_RGB = C I_lambda): a channel whose
    normalised sensitivity is the convex mix a s_R + (1 - a) s_B of two others
    sees the same mix of their transmittances exp(-mu_R) and exp(-mu_B)."""
    resp = np.asarray(spectra.response, dtype=np.float64)
    s = resp / resp.sum(axis=1, keepdims=True)
    mixed = np.stack([s[0], s[2], alpha * s[0] + (1 - alpha) * s[2]])
    m = orc.Model(spectra.eps_hb, spectra.eps_hbo2, mixed, spectra.path_length_cm)
    for hb, hbo2 in [(20.0, 90.0), (120.0, 60.0), (60.0, 0.0)]:
        T = np.exp(-orc.mu(m, hb, hbo2))
        assert abs(T[2] - (alpha * T[0] + (1 - alpha) * T[1])) <= 1e-14 * T[2]
        assert abs(T[0] - T[1]) > 1e-3
