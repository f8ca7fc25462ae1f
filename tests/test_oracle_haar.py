"""Pins of the oracle's 2D Haar transform (Method, Eq. 1-2 and Eq. 4)."""
import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import hb_oracle as orc
from tests.conftest import load_golden

# Mallat positions of [LL, D1, D2, D3] for a single 2x2 image.
POS = [(0, 0), (1, 0), (1, 1), (0, 1)]


def test_golden_matrix_is_orthogonal_and_symmetric():
    H = load_golden("haar_matrix_eq2.txt")
    assert np.allclose(H, H.T, atol=0)
    assert np.allclose(H @ H, np.eye(4), atol=1e-15)   # H = H^-1 (Eq. 4, "since H = H*")


def test_forward_reproduces_eq2_on_unit_windows():
    """Each unit window e_i must map to row i of H (Haar(I) = I * H)."""
    H = load_golden("haar_matrix_eq2.txt")
    order = [(0, 0), (0, 1), (1, 0), (1, 1)]   # {I(x,y), I(x,y+1), I(x+1,y), I(x+1,y+1)}, x = row
    for i, (r, c) in enumerate(order):
        x = np.zeros((2, 2))
        x[r, c] = 1.0
        co = orc.haar_forward(x, 1)
        got = np.array([co[p] for p in POS])
        assert np.array_equal(got, H[i]), (i, got, H[i])


def test_lowpass_row_matches_h_lp():
    hlp = load_golden("lowpass_row.txt")
    x = np.array([[1.0, 2.0], [3.0, 5.0]])
    co = orc.haar_forward(x, 1)
    assert co[0, 0] == pytest.approx(hlp @ np.array([1.0, 2.0, 3.0, 5.0]), abs=1e-15)


@pytest.mark.parametrize("levels", [0, 1, 2, 3, 4, 5])
def test_perfect_reconstruction_and_parseval(levels):
    rng = np.random.default_rng(levels)
    x = rng.normal(size=(64, 96)) + 3.0
    co = orc.haar_forward(x, levels)
    back = orc.haar_inverse(co, levels)
    assert np.max(np.abs(back - x)) <= 1e-14 * np.max(np.abs(x)) * 8
    assert np.sum(co ** 2) == pytest.approx(np.sum(x ** 2), rel=1e-13)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_ll_is_scaled_block_mean(levels):
    rng = np.random.default_rng(10 + levels)
    x = rng.uniform(0.1, 2.0, size=(32, 48))
    co = orc.haar_forward(x, levels)
    b = 1 << levels
    means = x.reshape(32 // b, b, 48 // b, b).mean(axis=(1, 3))
    ll = co[: 32 // b, : 48 // b]
    assert np.allclose(ll, b * means, rtol=1e-14, atol=0)   # LL_n = 2^n * block mean


@pytest.mark.parametrize("shape,levels", [((4, 4), 1), ((4, 4), 2), ((8, 8), 1), ((8, 8), 2),
                                          ((8, 8), 3), ((8, 4), 2), ((4, 8), 1)])
def test_matches_kronecker_brute_force(shape, levels):
    rng = np.random.default_rng(hash(shape) % 1000 + levels)
    x = rng.normal(size=shape)
    W = bf.haar_matrix(shape[0], shape[1], levels)
    assert np.allclose(W @ W.T, np.eye(W.shape[0]), atol=1e-14)
    co = orc.haar_forward(x, levels)
    assert np.allclose(co.reshape(-1), W @ x.reshape(-1), atol=1e-14)
    assert np.allclose(orc.haar_inverse(co, levels).reshape(-1), W.T @ co.reshape(-1), atol=1e-14)


def test_block_constant_has_zero_details():
    rng = np.random.default_rng(3)
    blocks = rng.normal(size=(4, 6))
    x = np.kron(blocks, np.ones((4, 4)))   # 16 x 24, constant on 4x4 blocks
    co = orc.haar_forward(x, 2)
    det = co.copy()
    det[:4, :6] = 0.0
    assert np.max(np.abs(det)) < 1e-14
