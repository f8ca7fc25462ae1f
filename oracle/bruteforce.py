"""Dense brute-force formulation of the path for tiny frames (numpy, FP64).

TEST INFRASTRUCTURE ONLY.  It pins the C oracle from an independent angle:
  - the n-level 2D Haar transform of an h x w frame is one explicit orthogonal
    matrix W built from Kronecker products of the 1-D Haar step (Method,
    Eq. 1-2: the 4x4 H is the Kronecker square of the 1-D step up to row order);
  - the Jacobian E of the forward model comes from a complex-step derivative;
  - the Tikhonov operator comes from least squares on the augmented system
    [E; sqrt(gamma) I] (Method, Eq. 5), not from the normal equations;
  - the posterior mean uses scipy's logsumexp;
  - the inverse transform is W transposed.
No code is shared with hb_oracle.c.
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp


def haar_step_1d(n: int) -> np.ndarray:
    """One level of the orthonormal 1-D Haar step on n samples: first n/2 rows
    are pairwise sums / sqrt(2), last n/2 rows pairwise (first - second) / sqrt(2)."""
    A = np.zeros((n, n))
    r = 1.0 / np.sqrt(2.0)
    for i in range(n // 2):
        A[i, 2 * i] = r
        A[i, 2 * i + 1] = r
        A[n // 2 + i, 2 * i] = r
        A[n // 2 + i, 2 * i + 1] = -r
    return A


def haar_matrix(h: int, w: int, levels: int) -> np.ndarray:
    """W such that vec(coefficients) = W vec(frame), row-major vec, Mallat layout."""
    W = np.eye(h * w)
    for l in range(levels):
        hh, ww = h >> l, w >> l
        step = np.kron(haar_step_1d(hh), haar_step_1d(ww))   # acts on the hh x ww sub-image
        # Embed: indices of the top-left hh x ww sub-image inside the h x w frame.
        idx = (np.arange(hh)[:, None] * w + np.arange(ww)[None, :]).reshape(-1)
        Lm = np.eye(h * w)
        Lm[np.ix_(idx, idx)] = step
        W = Lm @ W
    return W


def forward_model_mu(c: np.ndarray, eps_hb, eps_hbo2, response, path_cm) -> np.ndarray:
    """mu(c) for c [..., 2]; works with complex c (complex-step derivatives)."""
    resp = np.asarray(response, dtype=np.float64)
    resp = resp / resp.sum(axis=1, keepdims=True)
    c = np.asarray(c)
    att = np.exp(-path_cm * (c[..., 0:1] * np.asarray(eps_hb) + c[..., 1:2] * np.asarray(eps_hbo2)))
    return -np.log(att @ resp.T)


def jacobian_complex_step(c, eps_hb, eps_hbo2, response, path_cm, h: float = 1e-30) -> np.ndarray:
    E = np.zeros((3, 2))
    for i in range(2):
        cc = np.array(c, dtype=np.complex128)
        cc[i] += 1j * h
        E[:, i] = np.imag(forward_model_mu(cc, eps_hb, eps_hbo2, response, path_cm)) / h
    return E


def tikhonov_lstsq(E: np.ndarray, lambda_rel: float) -> np.ndarray:
    gamma = lambda_rel * np.trace(E.T @ E) / 2.0
    rows = E.shape[0]
    A = np.vstack([E, np.sqrt(gamma) * np.eye(2)])
    B = np.vstack([np.eye(rows), np.zeros((2, rows))])
    M, *_ = np.linalg.lstsq(A, B, rcond=None)
    return M


def grid_nodes(thb_min, thb_max, gt, so2_min, so2_max, gs, mu_fn):
    thb = np.linspace(thb_min, thb_max, gt)
    so2 = np.linspace(so2_min, so2_max, gs)
    T, S = np.meshgrid(thb, so2, indexing="ij")
    c = np.stack([T * (1 - S), T * S], axis=-1).reshape(-1, 2)
    return c, mu_fn(c)


def posterior_mean(c: np.ndarray, mu: np.ndarray, ybar: np.ndarray, sigma: float,
                   illumination: int = 0) -> np.ndarray:
    r = ybar[None, :] - mu
    if illumination:
        # integrating a flat prior over b*(1,1,1) leaves the residual's
        # component orthogonal to (1,1,1): the projector I - 11'/3
        r = r @ (np.eye(3) - np.full((3, 3), 1.0 / 3.0))
    ll = -np.sum(r ** 2, axis=1) / (2.0 * sigma ** 2)
    lw = ll - logsumexp(ll)
    return np.exp(lw) @ c


def estimate(frames: np.ndarray, levels: int, spectra, grid: dict, lambda_rel: float,
             sigma: float, floor: float = 1e-4, ref=None, lowpass: int = 0,
             thb_eps: float = 1e-3, illumination: int = 0) -> np.ndarray:
    """frames [H][W][3] -> maps [4][H][W]."""
    eps_hb, eps_hbo2, response, path_cm = spectra
    h, w, _ = frames.shape
    mu_fn = lambda c: forward_model_mu(c, eps_hb, eps_hbo2, response, path_cm)
    if ref is None:
        thb_c = 0.5 * (grid["thb_min"] + grid["thb_max"])
        so2_c = 0.5 * (grid["so2_min"] + grid["so2_max"])
        ref = (thb_c * (1 - so2_c), thb_c * so2_c)
    E = jacobian_complex_step(ref, eps_hb, eps_hbo2, response, path_cm)
    M = tikhonov_lstsq(E, lambda_rel)
    W = haar_matrix(h, w, levels)
    y = -np.log(np.maximum(frames.astype(np.float64), floor))           # [H][W][3]
    coef = np.stack([W @ y[:, :, k].reshape(-1) for k in range(3)], axis=1)   # [HW][3]
    hl, wl = h >> levels, w >> levels
    ll_idx = (np.arange(hl)[:, None] * w + np.arange(wl)[None, :]).reshape(-1)
    is_ll = np.zeros(h * w, dtype=bool)
    is_ll[ll_idx] = True
    conc = coef @ M.T                                                   # Tikhonov on all
    scale = 2.0 ** levels
    if lowpass == 0:
        cg, mug = grid_nodes(grid["thb_min"], grid["thb_max"], grid["grid_thb"],
                             grid["so2_min"], grid["so2_max"], grid["grid_so2"], mu_fn)
        for i in ll_idx:
            conc[i] = scale * posterior_mean(cg, mug, coef[i] / scale, sigma, illumination)
    else:
        mref = mu_fn(np.asarray(ref))
        for i in ll_idx:
            conc[i] = scale * (np.asarray(ref) + M @ (coef[i] / scale - mref))
    x = W.T @ conc                                                      # [HW][2]
    hb, hbo2 = x[:, 0].reshape(h, w), x[:, 1].reshape(h, w)
    thb = hb + hbo2
    with np.errstate(invalid="ignore", divide="ignore"):
        so2 = np.where(thb > thb_eps, hbo2 / thb, np.nan)
    return np.stack([hb, hbo2, thb, so2])
