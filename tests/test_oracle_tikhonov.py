"""Pins of the oracle's Tikhonov operator (Method, Eq. 5, with C -> E)."""
import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import hb_oracle as orc


@pytest.fixture
def E(model):
    return orc.jacobian(model, 38.5, 71.5)


def test_normal_equations(E):
    M, gamma = orc.tikhonov(E, 1e-3)
    A = E.T @ E + gamma * np.eye(2)
    assert np.max(np.abs(A @ M - E.T)) <= 1e-13 * np.max(np.abs(E))


def test_gamma_is_relative_to_trace(E):
    _, gamma = orc.tikhonov(E, 0.25)
    assert gamma == pytest.approx(0.25 * np.trace(E.T @ E) / 2, rel=1e-15)


@pytest.mark.parametrize("lam", [0.0, 1e-6, 1e-3, 0.1, 10.0])
def test_matches_augmented_least_squares(E, lam):
    M, _ = orc.tikhonov(E, lam)
    assert np.allclose(M, bf.tikhonov_lstsq(E, lam), rtol=1e-10, atol=0)


def test_lambda_to_zero_recovers_consistent_data(E):
    c = np.array([42.0, 87.0])
    M, _ = orc.tikhonov(E, 0.0)
    assert np.allclose(M @ (E @ c), c, rtol=1e-10)
    # and the regularised solution converges to it as lambda -> 0
    errs = [np.abs(orc.tikhonov(E, lam)[0] @ (E @ c) - c).max() for lam in (1e-2, 1e-4, 1e-6)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3 * np.abs(c).max()


def test_square_system_is_exact_inverse():
    E2 = np.array([[0.31, 0.12], [0.05, 0.44]])
    M, _ = orc.tikhonov(E2, 0.0)
    assert np.allclose(M, np.linalg.inv(E2), rtol=1e-13)


def test_singular_system_is_rejected():
    Es = np.array([[1.0, 2.0], [2.0, 4.0], [3.0, 6.0]])
    with pytest.raises(np.linalg.LinAlgError):
        orc.tikhonov(Es, 0.0)


def test_regularisation_shrinks(E):
    norms = [np.linalg.norm(orc.tikhonov(E, lam)[0]) for lam in (0.0, 1e-2, 1.0, 100.0)]
    assert all(a > b for a, b in zip(norms, norms[1:]))
