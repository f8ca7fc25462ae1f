"""Pins of the oracle's posterior mean on the low-pass band."""
import numpy as np
import pytest
from scipy import stats

from oracle import bruteforce as bf
from oracle import hb_oracle as orc


def _params(**kw):
    base = dict(width=2, height=2, grid_thb=32, grid_so2=32, thb_min=20, thb_max=200,
                so2_min=0.3, so2_max=1.0, sigma=0.01)
    base.update(kw)
    return orc.Params(**base)


def test_one_node_grid_returns_the_node(model):
    p = _params(grid_thb=1, grid_so2=1, thb_min=77.0, so2_min=0.41)
    c, mu = orc.grid(p, model)
    out = orc.posterior_mean(c, mu, [0.3, -0.2, 0.9], 0.01)
    assert np.array_equal(out, c[0])


def test_two_node_grid_is_a_logistic(model):
    """Two hypotheses with equal prior: the posterior weight of node 2 is the
    logistic function of the log-likelihood ratio of two Gaussians."""
    p = _params(grid_thb=2, grid_so2=1, thb_min=60.0, thb_max=90.0, so2_min=0.7)
    c, mu = orc.grid(p, model)
    rng = np.random.default_rng(0)
    for sigma in (0.003, 0.01, 0.05):
        for _ in range(5):
            y = 0.5 * (mu[0] + mu[1]) + rng.normal(0, 0.01, 3)
            llr = (np.sum((y - mu[0]) ** 2) - np.sum((y - mu[1]) ** 2)) / (2 * sigma ** 2)
            p2 = 1.0 / (1.0 + np.exp(-llr))
            want = c[0] + (c[1] - c[0]) * p2
            got = orc.posterior_mean(c, mu, y, sigma)
            assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_infinite_sigma_gives_grid_mean(model):
    p = _params(grid_thb=17, grid_so2=9)
    c, mu = orc.grid(p, model)
    out = orc.posterior_mean(c, mu, mu[5], 1e8)
    thb_mean, so2_mean = 0.5 * (20 + 200), 0.5 * (0.3 + 1.0)   # inclusive linspace means
    assert np.allclose(out, [thb_mean * (1 - so2_mean), thb_mean * so2_mean], rtol=1e-9)


def test_truncated_normal_posterior(spectra):
    """Linear forward model (one wavelength per channel) and a 1-D THb grid at
    fixed SO2: the posterior of THb is a normal truncated to the grid range."""
    n = spectra.eps_hb.size
    picks = [10, 28, 45]
    resp = np.zeros((3, n))
    for k, j in enumerate(picks):
        resp[k, j] = 1.0
    m = orc.Model(spectra.eps_hb, spectra.eps_hbo2, resp, 0.1)
    s0 = 0.6
    e = np.array([0.1 * ((1 - s0) * spectra.eps_hb[j] + s0 * spectra.eps_hbo2[j]) for j in picks])
    p = _params(grid_thb=20001, grid_so2=1, so2_min=s0)
    c, mu = orc.grid(p, m)
    rng = np.random.default_rng(5)
    for m0, sd in [(195.0, 10.0), (30.0, 6.0), (110.0, 4.0)]:
        sigma = sd * np.linalg.norm(e)
        # observation whose least-squares THb is m0, plus an orthogonal component
        orth = np.cross(e, rng.normal(size=3))
        y = m0 * e + 0.01 * orth / np.linalg.norm(orth)
        a, b = (20.0 - m0) / sd, (200.0 - m0) / sd
        thb_mean = stats.truncnorm.mean(a, b, loc=m0, scale=sd)
        got = orc.posterior_mean(c, mu, y, sigma)
        assert got[0] == pytest.approx((1 - s0) * thb_mean, abs=1e-2)
        assert got[1] == pytest.approx(s0 * thb_mean, abs=1e-2)


@pytest.mark.parametrize("sigma", [1e-2, 1e-3, 1e-4])
def test_grid_aligned_truth_converges(model, spectra, sigma):
    p = _params(grid_thb=64, grid_so2=64)
    c, mu = orc.grid(p, model)
    gstar = 37 * 64 + 21
    cstar = c[gstar]
    y = bf.forward_model_mu(cstar, spectra.eps_hb, spectra.eps_hbo2, spectra.response,
                            spectra.path_length_cm)
    got = orc.posterior_mean(c, mu, y, sigma)
    ll = -np.sum((y - mu) ** 2, axis=1) / (2 * sigma ** 2)
    w = np.exp(ll - ll[gstar])
    w[gstar] = 0.0
    bound = np.sum(w[:, None] * np.abs(c - cstar), axis=0) / (1.0 + w.sum())
    assert np.all(np.abs(got - cstar) <= bound + 1e-9)
    if sigma <= 1e-3:
        assert np.max(np.abs(got - cstar)) < 0.05


def test_matches_logsumexp_brute_force(model):
    rng = np.random.default_rng(11)
    p = _params(grid_thb=24, grid_so2=20)
    c, mu = orc.grid(p, model)
    for sigma in (0.005, 0.01, 0.03):
        for _ in range(10):
            y = mu[rng.integers(len(mu))] + rng.normal(0, 0.02, 3)
            assert np.allclose(orc.posterior_mean(c, mu, y, sigma), bf.posterior_mean(c, mu, y, sigma),
                               rtol=1e-11, atol=1e-11)


def test_nan_observation_propagates(model):
    c, mu = orc.grid(_params(grid_thb=4, grid_so2=4), model)
    out = orc.posterior_mean(c, mu, [np.nan, 0.1, 0.2], 0.01)
    assert np.all(np.isnan(out))


def test_illumination_term_is_a_marginal_over_a_log_offset(model):
    """Integrating exp(-|ybar - mu_g - b (1,1,1)|^2 / (2 sigma^2)) over b (flat
    prior; numerical quadrature) gives the weights of the illumination term."""
    from scipy.integrate import quad
    p = _params(grid_thb=5, grid_so2=4)
    c, mu = orc.grid(p, model)
    rng = np.random.default_rng(21)
    sigma = 0.02
    for _ in range(3):
        y = mu[rng.integers(len(mu))] + rng.normal(0, 0.03, 3) + 0.2
        lw = []
        for g in range(len(mu)):
            d = y - mu[g]
            b0 = d.mean()   # centre the integral on the maximising offset
            val, _ = quad(lambda b: np.exp(-np.sum((d - b) ** 2) / (2 * sigma ** 2) +
                                           np.sum((d - b0) ** 2) / (2 * sigma ** 2)), b0 - 1, b0 + 1,
                          points=[b0], epsabs=0, epsrel=1e-12, limit=200)
            lw.append(np.log(val) - np.sum((d - b0) ** 2) / (2 * sigma ** 2))
        lw = np.array(lw)
        w = np.exp(lw - lw.max())
        want = (w[:, None] * c).sum(0) / w.sum()
        got = orc.posterior_mean(c, mu, y, sigma, illumination=1)
        assert np.allclose(got, want, rtol=1e-8, atol=1e-8)


def test_illumination_term_is_offset_invariant(model):
    p = _params(grid_thb=20, grid_so2=16)
    c, mu = orc.grid(p, model)
    y = mu[77] + np.array([0.003, -0.002, 0.004])
    a = orc.posterior_mean(c, mu, y, 0.01, illumination=1)
    for b in (-0.3, 0.05, 0.7):
        assert np.allclose(orc.posterior_mean(c, mu, y + b, 0.01, illumination=1), a, rtol=1e-12, atol=1e-12)
    # without the term an offset moves the estimate
    assert not np.allclose(orc.posterior_mean(c, mu, y + 0.05, 0.01), orc.posterior_mean(c, mu, y, 0.01), atol=1e-3)
