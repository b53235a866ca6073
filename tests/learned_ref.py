"""The learned-weight oracle applied to the GPU's own records (test infrastructure).

The HIP learned filter and training step read the records of a gather; the
oracle's float64 features, MLP, set softmax and backward are evaluated on the
same records (colours and rho as stored in binary16), with the MLP weights
exactly as the device holds them (bfloat16 weights, float32 biases and
standardisation).
"""
from __future__ import annotations

import numpy as np

from oracle import learned

from tests.parity import f16_to_f64

OFF_B3, OFF_MEAN, OFF_INV = 128, 132, 140


def records_subset(g_off, g_ids, g_crho, pixels):
    """CSR sub-arrays of the sets of `pixels` (indices into the frame)."""
    counts = np.diff(g_off)[pixels]
    starts = g_off[pixels]
    sel = (np.concatenate([np.arange(s, s + c) for s, c in zip(starts, counts)])
           if counts.sum() else np.zeros(0, np.int64))
    off = np.zeros(len(pixels) + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    return off, g_ids[sel], g_crho[sel]


def raw_features(off, ids, crho, pixels, f, dep, cams, fx, fy, cx, cy, window, radius):
    seg = np.repeat(np.arange(len(pixels)), np.diff(off))
    col = f16_to_f64(crho[:, :3].copy())
    rho = f16_to_f64(crho[:, 3].copy())
    x = learned.features(seg, ids, rho, col, off, np.asarray(pixels), f, dep, cams, fx, fy, cx, cy,
                         window, radius)
    return x, col


def oracle_mlp_from_device(params) -> learned.MLP:
    """The oracle MLP holding the device's stored values."""
    w1, b1, w2, b2, w3, b3 = params.weights_f64()
    b = params.b.cpu().numpy().astype(np.float64)
    return learned.MLP(w1, b1, w2, b2, w3, b3, b[OFF_MEAN:OFF_MEAN + 8].copy(),
                       1.0 / b[OFF_INV:OFF_INV + 8])


def random_mlp(seed: int, mean, std, bias_scale=0.3, out_scale=3.0) -> learned.MLP:
    """He-initialised MLP with non-zero biases and a wide logit range."""
    m = learned.init_mlp(seed, mean, std)
    rng = np.random.default_rng(seed + 1)
    m.b1 = rng.normal(size=64) * bias_scale
    m.b2 = rng.normal(size=64) * bias_scale
    m.w3 = m.w3 * out_scale
    m.b3 = 0.25
    return m


def learned_filter(x_raw, col, off, c_ref, mlp: learned.MLP):
    xs = learned.standardise(x_raw, mlp)
    m, _ = learned.forward(xs, mlp)
    o, _ = learned.set_softmax_mean(m, col, off, c_ref)
    return o
