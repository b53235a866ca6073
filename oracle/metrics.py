"""Image quality metric (test infrastructure only).

PSNR as plotted for denoising in Sec. 5 (the denoising PSNR figure): on the
0-1 scale, PSNR = 10 log10(1 / MSE) over all pixels and channels, which equals
20 log10(255 / sigma) for zero-mean error of standard deviation sigma on the
0-255 scale.
"""
from __future__ import annotations

import numpy as np


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(1.0 / mse)
