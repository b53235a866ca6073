"""Camera matrices and relative transforms (test infrastructure only).

C^f is the camera-to-world 4x4 matrix of frame f (Sec. 3: samples are formed
by projecting a pixel with its camera matrix and depth). Sec. 4 Eq. 2 maps a
pixel of input frame J back into the output view with C_O . C_J^{-1}; the
depth-guided gather does the opposite direction, output view -> frame J, with
T_{J<-f} = (C^J)^{-1} . C^f. Here the inverse is a general 4x4 inverse (LAPACK
through numpy), and J = f yields exactly the identity.
"""
from __future__ import annotations

import numpy as np


def intrinsics(fx: float, fy: float, cx: float, cy: float) -> np.ndarray:
    return np.array([[fx, 0.0, cx], [0.0, fy, cy], [0.0, 0.0, 1.0]], dtype=np.float64)


def relative(c_f: np.ndarray, c_j: np.ndarray, same_frame: bool) -> np.ndarray:
    """T_{J<-f} = inv(C^J) @ C^f as a 4x4 float64 matrix (identity when J == f)."""
    if same_frame:
        return np.eye(4, dtype=np.float64)
    return np.linalg.inv(np.asarray(c_j, dtype=np.float64)) @ np.asarray(c_f, dtype=np.float64)
