"""Sample-set filtering (test infrastructure only).

Sec. 5 Eq. 3: O(p) = (1 / W) sum_{s in S(p)} w(s) s_rgb with W = sum w(s).
Sec. 5.1 Eq. 4: the denoising weight is a Gaussian around the reference
sample s_ref (the sample that the output pixel itself contributes: frame f,
pixel p) with a diagonal covariance. Here the terms are
  w(s) = exp(-rho_s^2 / (2 sd^2)) * exp(-|c_s - c_ref|^2 / (2 sc^2)) * exp(-(J_s - f)^2 / (2 st^2))
where rho_s is the sample's relative depth residual (the depth-guided gather's
stand-in for the scene-space distance to s_ref), c_ref = I^f(p), and a sigma
of +inf disables its term (weight factor 1). sd alone is the depth-Gaussian
weighted mean; sd = sc = st = inf is the plain mean of Sec. 5.1 (w = 1).
An empty set returns the input colour I^f(p) (reading: the paper is silent).
"""
from __future__ import annotations

import math

import numpy as np

from .gather import ID_SHIFT, OracleSets


def _factor(dist2: np.ndarray, sigma: float) -> np.ndarray:
    if math.isinf(sigma):
        return np.ones_like(dist2)
    return np.exp(-dist2 / (2.0 * sigma * sigma))


def weighted_mean(offsets: np.ndarray, colour: np.ndarray, rho: np.ndarray, dj: np.ndarray,
                  c_ref: np.ndarray, sigma_d: float, sigma_c: float = math.inf,
                  sigma_t: float = math.inf) -> np.ndarray:
    """Eq. 3 with the weight above over CSR sets; returns [n, 3] float64."""
    n = offsets.size - 1
    counts = np.diff(offsets)
    seg = np.repeat(np.arange(n), counts)
    dc2 = np.sum((colour - c_ref[seg]) ** 2, axis=1)
    w = _factor(rho * rho, sigma_d) * _factor(dc2, sigma_c) * _factor(dj.astype(np.float64) ** 2, sigma_t)
    wsum = np.bincount(seg, weights=w, minlength=n)
    out = np.empty((n, 3))
    for ch in range(3):
        out[:, ch] = np.bincount(seg, weights=w * colour[:, ch], minlength=n)
    empty = counts == 0
    with np.errstate(invalid="ignore", divide="ignore"):
        out = out / wsum[:, None]
    out[empty] = c_ref[empty]
    return out


def filter_sets(sets: OracleSets, colour_f: np.ndarray, window: int, sigma_d: float,
                sigma_c: float = math.inf, sigma_t: float = math.inf) -> np.ndarray:
    """Filter the oracle's own sets; colour_f is the frame-f colour plane [H, W, 3]."""
    c_ref = colour_f.reshape(-1, 3)[sets.pixels]
    dj = (sets.ids.astype(np.int64) >> ID_SHIFT) - window
    return weighted_mean(sets.offsets, sets.colour, sets.rho, dj, c_ref, sigma_d, sigma_c, sigma_t)


def sample_weight_sum(sets: OracleSets, sigma_d: float) -> np.ndarray:
    """W(p) of Eq. 3 for the depth term alone (used for the W/|S| statistic of Sec. 5)."""
    n = sets.offsets.size - 1
    seg = np.repeat(np.arange(n), np.diff(sets.offsets))
    return np.bincount(seg, weights=_factor(sets.rho ** 2, sigma_d), minlength=n)
