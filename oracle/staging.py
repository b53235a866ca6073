"""Storage rounding of the input planes (test infrastructure only).

Colour arrives as 8-bit RGB on the 0-255 scale and is kept on the 0-1 scale
(the paper works on 0-255; a sample colour here is that value divided by 255).
Depth arrives as float32 z-depth. Mode Q rounds both to IEEE binary16 (round
to nearest, ties to even) and widens the result exactly to float64.
"""
from __future__ import annotations

import numpy as np


def colour_q(rgb_u8: np.ndarray) -> np.ndarray:
    """u8 RGB -> binary16(c / 255) as float64, same shape."""
    return (rgb_u8.astype(np.float64) / 255.0).astype(np.float16).astype(np.float64)


def depth_q(depth_f32: np.ndarray) -> np.ndarray:
    """float32 depth -> binary16 depth as float64 (values above 65504 become inf)."""
    with np.errstate(over="ignore"):
        return depth_f32.astype(np.float64).astype(np.float16).astype(np.float64)


def colour_f(rgb_u8: np.ndarray) -> np.ndarray:
    """u8 RGB -> c / 255 in float64 (mode F, no storage rounding)."""
    return rgb_u8.astype(np.float64) / 255.0


def depth_f(depth_f32: np.ndarray) -> np.ndarray:
    return depth_f32.astype(np.float64)
