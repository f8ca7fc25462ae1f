"""End-to-end pins of the oracle: brute force, commutation, invariants."""
import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import hb_oracle as orc
from paper_1706_07263_amd import synth

GRID = dict(grid_thb=12, grid_so2=10, thb_min=20.0, thb_max=200.0, so2_min=0.3, so2_max=1.0)


def _frame(h, w, seed, sp):
    fr, _, _ = synth.single_frame(h, w, config=90, stream=seed, sp=sp)
    return fr.astype(np.float64)


@pytest.mark.parametrize("shape,levels,lowpass", [((4, 4), 1, 0), ((4, 4), 2, 0), ((8, 8), 1, 0),
                                                  ((8, 8), 2, 0), ((8, 8), 3, 0), ((4, 8), 1, 1),
                                                  ((8, 8), 2, 1)])
def test_matches_dense_brute_force(spectra, model, shape, levels, lowpass):
    fr = _frame(*shape, seed=levels + 3 * lowpass, sp=spectra)
    p = orc.Params(width=shape[1], height=shape[0], levels=levels, lowpass=lowpass, **GRID)
    got = orc.estimate(p, model, fr)[0]
    want = bf.estimate(fr, levels, (spectra.eps_hb, spectra.eps_hbo2, spectra.response,
                                    spectra.path_length_cm), GRID, 1e-3, 0.01, lowpass=lowpass)
    assert np.allclose(got, want, rtol=0, atol=1e-11), np.max(np.abs(got - want))


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_tikhonov_lowpass_commutes_with_haar(spectra, model, levels):
    """With Tikhonov on every band the path is one affine map per pixel,
    c(p) = c_ref + M (y(p) - mu(c_ref)): the spectral inverse commutes with the
    spatial Haar transform (Method, Eq. 3)."""
    fr = _frame(16, 24, seed=7, sp=spectra)
    p = orc.Params(width=24, height=16, levels=levels, lowpass=1, **GRID)
    got = orc.estimate(p, model, fr)[0]
    ref = np.array(p.ref())
    E = orc.jacobian(model, *ref)
    M, _ = orc.tikhonov(E, 1e-3)
    y = -np.log(fr)
    want = ref[:, None, None] + np.einsum("ij,hwj->ihw", M, y - orc.mu(model, *ref))
    assert np.allclose(got[:2], want, rtol=0, atol=1e-10)


@pytest.mark.parametrize("levels", [1, 2])
def test_block_constant_frame(spectra, model, levels):
    """A frame constant on each 2^n block has no directional content: the output
    is constant per block and equals the posterior mean of that block."""
    b = 1 << levels
    rng = np.random.default_rng(2)
    small = rng.uniform(0.3, 0.9, size=(16 // b, 16 // b, 3))
    fr = np.kron(small, np.ones((b, b, 1)))
    p = orc.Params(width=16, height=16, levels=levels, **GRID)
    out = orc.estimate(p, model, fr)[0]
    c, mu = orc.grid(p, model)
    for (i, j) in [(0, 0), (1, 2), (16 // b - 1, 16 // b - 1)]:
        pm = orc.posterior_mean(c, mu, -np.log(small[i, j]), 0.01)
        blk = out[:2, i * b:(i + 1) * b, j * b:(j + 1) * b]
        assert np.allclose(blk, pm[:, None, None], rtol=0, atol=1e-10)


def test_illumination_offset_only_moves_lowpass(spectra, model):
    """Scaling all intensities of one block by a common factor adds a constant
    log offset (the paper's global-illumination term, before Eq. 9): the
    directional part of the output is unchanged, so the output moves by one
    constant per map within that block."""
    fr = _frame(8, 8, seed=4, sp=spectra)
    fr2 = fr.copy()
    fr2[2:4, 4:6] *= 0.93
    p = orc.Params(width=8, height=8, levels=1, **GRID)
    a = orc.estimate(p, model, fr)[0]
    b = orc.estimate(p, model, fr2)[0]
    d = (b - a)[:2, 2:4, 4:6]
    assert np.allclose(d, d[:, :1, :1], atol=1e-10)
    other = np.ones((8, 8), bool)
    other[2:4, 4:6] = False
    assert np.allclose(a[:, other], b[:, other], atol=0, rtol=0, equal_nan=True)


def test_crop_equals_full_frame(spectra, model):
    """Blocks are independent: an aligned crop gives the same values."""
    fr = _frame(32, 32, seed=5, sp=spectra)
    p = orc.Params(width=32, height=32, levels=2, **GRID)
    full = orc.estimate(p, model, fr)[0]
    pc = orc.Params(width=8, height=12, levels=2, **GRID)
    crop = orc.estimate(pc, model, fr[8:20, 16:24])[0]
    assert np.array_equal(crop, full[:, 8:20, 16:24])


def test_maps_and_so2_nan_below_threshold(model):
    p = orc.Params(width=4, height=4, levels=1, lowpass=1, ref_hb=0.0, ref_hbo2=0.0, **GRID)
    fr = np.ones((4, 4, 3))                        # zero attenuation -> zero concentration
    out = orc.estimate(p, model, fr)[0]
    assert np.max(np.abs(out[:3])) < 1e-9
    assert np.all(np.isnan(out[3]))
    p2 = orc.Params(width=4, height=4, levels=1, **GRID)
    fr2 = np.full((4, 4, 3), 0.5)
    o2 = orc.estimate(p2, model, fr2)[0]
    assert np.allclose(o2[2], o2[0] + o2[1], rtol=0, atol=0)
    assert np.allclose(o2[3], o2[1] / o2[2], rtol=1e-15)


def test_floor_clamp_and_nan_propagation(model):
    p = orc.Params(width=4, height=4, levels=1, **GRID)
    fr = np.full((4, 4, 3), 0.6)
    fr2 = fr.copy()
    fr2[0, 0, 1] = -0.2                              # clamps to the floor
    fr3 = fr.copy()
    fr3[0, 0, 1] = p.floor
    assert np.array_equal(orc.estimate(p, model, fr2), orc.estimate(p, model, fr3), equal_nan=True)
    fr4 = fr.copy()
    fr4[2, 3, 0] = np.nan
    out = orc.estimate(p, model, fr4)[0]
    assert np.all(np.isnan(out[:, 2:4, 2:4]))        # the whole 2x2 block
    assert not np.any(np.isnan(out[:, :2, :]))


def test_rejects_non_divisible_shape(model):
    p = orc.Params(width=6, height=4, levels=2, **GRID)
    with pytest.raises(ValueError):
        orc.estimate(p, model, np.full((4, 6, 3), 0.5))


def test_illumination_term_makes_block_gain_invisible(spectra, model):
    """With the illumination term a common gain on all intensities of a block
    (a constant log offset in every channel and pixel) changes nothing."""
    fr = _frame(8, 8, seed=6, sp=spectra)
    fr2 = fr.copy()
    fr2[2:4, 4:6] *= 0.8
    fr2[0:2, 0:2] *= 1.1
    p = orc.Params(width=8, height=8, levels=1, illumination=1, **GRID)
    a = orc.estimate(p, model, fr)[0]
    b = orc.estimate(p, model, fr2)[0]
    assert np.allclose(a, b, rtol=0, atol=1e-9, equal_nan=True)


@pytest.mark.parametrize("levels", [1, 2])
def test_illumination_term_matches_dense_brute_force(spectra, model, levels):
    fr = _frame(8, 8, seed=8 + levels, sp=spectra)
    p = orc.Params(width=8, height=8, levels=levels, illumination=1, **GRID)
    got = orc.estimate(p, model, fr)[0]
    want = bf.estimate(fr, levels, (spectra.eps_hb, spectra.eps_hbo2, spectra.response,
                                    spectra.path_length_cm), GRID, 1e-3, 0.01, illumination=1)
    assert np.allclose(got, want, rtol=0, atol=1e-11)
