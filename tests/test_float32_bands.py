"""The float32 error of the kernels' projections, measured at 1920x1080 with the
full-scale workload's observed camera poses, against the widths of the oracle's
comparison bands.

The kernels fold each relative pose with K into a float32 map in float64 and then
project in float32 with fused multiply-adds; the oracle projects in float64. A band
exempts decisions that this error could flip, so it must be wider than the error:
each test asserts the measured maximum stays at or below a fifth of its band.
The float32 arithmetic is modelled in numpy: each fused multiply-add is evaluated
exactly in float64 and rounded once more to float32 (within one float32 ulp of the
fused result), and the gather's approximate reciprocal is bounded by one ulp on
top of the correctly rounded one. Source depths are the scene's noise-free depths
with the workload's noise and outliers, stored as binary16.
"""
import math

import numpy as np
import pytest
import torch

from oracle import depth as odepth
from oracle import frustum as ofrustum
from oracle import gather as ogather
from scenegen import configs
from scenegen.scene import scene_setup, true_depth

N_SAMPLES = 20000


@pytest.fixture(scope="module")
def scene():
    wl = configs.full_scale()
    su = scene_setup(wl.spec)
    return wl, su


def _depths(wl, su, frame, pixels, seed):
    d = true_depth(wl.spec, su, frame, torch.as_tensor(pixels)).numpy()
    rng = np.random.default_rng(seed)
    d = d * (1.0 + wl.spec.depth_noise * rng.standard_normal(d.size))
    out = rng.random(d.size) < wl.spec.outlier_frac
    d[out] = 2.0 + 18.0 * rng.random(out.sum())
    return d.astype(np.float16).astype(np.float64)


def _k(wl):
    fx = wl.spec.focal
    return fx, fx, (wl.spec.width - 1) / 2.0, (wl.spec.height - 1) / 2.0


def _folded_map(a_to_b, fx, fy, cx, cy):
    """float32 M = K R K^-1 (3 x 3) and k = K t of a rigid map, folded in float64."""
    k = np.array([[fx, 0, cx], [0, fy, cy], [0, 0, 1.0]])
    m = k @ a_to_b[:3, :3] @ np.linalg.inv(k)
    t = k @ a_to_b[:3, 3]
    return m.astype(np.float32), t.astype(np.float32)


def _fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def _project32(m, t, x, y, d):
    """Y = d (M (x, y, 1)) + k in float32, the kernels' order of operations."""
    x, y, d = x.astype(np.float32), y.astype(np.float32), d.astype(np.float32)
    rows = []
    for i in range(3):
        a = _fma32(np.float32(m[i, 0]), x, _fma32(np.float32(m[i, 1]), y, np.full_like(x, m[i, 2])))
        rows.append(_fma32(d, a, np.full_like(x, t[i])))
    return rows


def _project64(c_from, c_to, x, y, d, fx, fy, cx, cy):
    """World-frame float64 reference: X = C_from [d K^-1 (x, y, 1), 1], Y = C_to^-1 X."""
    xc = np.stack([d * (x - cx) / fx, d * (y - cy) / fy, d, np.ones_like(d)])
    yw = np.linalg.inv(c_to) @ (c_from @ xc)
    z = yw[2]
    return fx * yw[0] / z + cx, fy * yw[1] / z + cy, z


def _sample_pixels(wl, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, wl.spec.width * wl.spec.height, N_SAMPLES)


def test_gather_projection_error_within_bands(scene):
    """Depth-guided gather: rounding band 2^-8 px on u, v; depth band 1e-5 on rho
    (relative z error); at output frame 150 of the 1080p +-50 workload, every
    fifth window frame."""
    wl, su = scene
    fx, fy, cx, cy = _k(wl)
    c2w = su.noisy.numpy()
    f = 150
    pix = _sample_pixels(wl, 1)
    x, y = (pix % wl.spec.width).astype(np.float64), (pix // wl.spec.width).astype(np.float64)
    d = _depths(wl, su, f, pix, 2)
    max_du, max_dz = 0.0, 0.0
    for j in range(f - wl.window, f + wl.window + 1, 5):
        if j == f:
            continue
        m, t = _folded_map(np.linalg.inv(c2w[j]) @ c2w[f], fx, fy, cx, cy)
        y0, y1, z = _project32(m, t, x, y, d)
        u64, v64, z64 = _project64(c2w[f], c2w[j], x, y, d, fx, fy, cx, cy)
        ok = (z64 > 1.0) & (np.abs(u64) < 3 * wl.spec.width) & (np.abs(v64) < 3 * wl.spec.height)
        inv = (np.float32(1.0) / z).astype(np.float32)
        u32 = y0.astype(np.float64) * inv.astype(np.float64)
        v32 = y1.astype(np.float64) * inv.astype(np.float64)
        # one ulp of the approximate reciprocal on top of the rounded quotient, and
        # half an ulp of the rounded u + 1/2 that the kernel floors
        ulp = np.maximum(np.abs(u32), np.abs(v32)) * (2.0 ** -23 + 2.0 ** -24)
        du = np.maximum(np.abs(u32 - u64), np.abs(v32 - v64)) + ulp
        max_du = max(max_du, float(du[ok].max()))
        max_dz = max(max_dz, float((np.abs(z.astype(np.float64) - z64) / z64)[ok].max()))
    print(f"gather: max |du| {max_du:.3g} px (band {ogather.EPS_PX:.3g}), max |dz|/z {max_dz:.3g}"
          f" (band {ogather.RHO_BAND:.3g})")
    assert max_du <= ogather.EPS_PX / 5
    assert max_dz <= ogather.RHO_BAND / 5


def test_frustum_carry_error_within_bands(scene):
    """Frustum gather: every source pixel carried into the output view in float32;
    L1 error of p' against the L1 band, relative z' error against the depth-range
    band; output frame 72 with a +-10 window (the benchmark's frustum leg)."""
    wl, su = scene
    fx, fy, cx, cy = _k(wl)
    c2w = su.noisy.numpy()
    f = 72
    max_l1, max_dz = 0.0, 0.0
    for j in range(f - 10, f + 11):
        if j == f:
            continue
        pix = _sample_pixels(wl, 100 + j)
        x, y = (pix % wl.spec.width).astype(np.float64), (pix // wl.spec.width).astype(np.float64)
        d = _depths(wl, su, j, pix, 200 + j)
        m, t = _folded_map(np.linalg.inv(c2w[f]) @ c2w[j], fx, fy, cx, cy)
        y0, y1, z = _project32(m, t, x, y, d)
        px = (y0 / z).astype(np.float64)    # correctly rounded float32 quotients
        py = (y1 / z).astype(np.float64)
        u64, v64, z64 = _project64(c2w[j], c2w[f], x, y, d, fx, fy, cx, cy)
        ok = (z64 > 1.0) & (np.abs(u64) < 3 * wl.spec.width) & (np.abs(v64) < 3 * wl.spec.height)
        max_l1 = max(max_l1, float((np.abs(px - u64) + np.abs(py - v64))[ok].max()))
        max_dz = max(max_dz, float((np.abs(z.astype(np.float64) - z64) / z64)[ok].max()))
    print(f"frustum: max L1 error {max_l1:.3g} px (band {ofrustum.L1_BAND:.3g}), max |dz'|/z' {max_dz:.3g}"
          f" (band {ofrustum.Z_BAND:.3g})")
    assert max_l1 <= ofrustum.L1_BAND / 5
    assert max_dz <= ofrustum.Z_BAND / 5


def test_depth_estimate_projection_error_within_band(scene):
    """Depth estimate: each hypothesis projected into the frames of a +-2 window and
    rounded; 32 hypotheses uniform in inverse depth over 1-30 m (the benchmark's
    depth leg), output frame 72; rounding band RND_BAND."""
    wl, su = scene
    fx, fy, cx, cy = _k(wl)
    c2w = su.noisy.numpy()
    f = 72
    hyp = (1.0 / np.linspace(1.0, 1.0 / 30.0, 32)).astype(np.float32).astype(np.float64)
    pix = _sample_pixels(wl, 7)[:4000]
    x, y = (pix % wl.spec.width).astype(np.float64), (pix // wl.spec.width).astype(np.float64)
    max_du = 0.0
    for j in (f - 2, f - 1, f + 1, f + 2):
        m, t = _folded_map(np.linalg.inv(c2w[j]) @ c2w[f], fx, fy, cx, cy)
        for dh in hyp:
            d = np.full(x.shape, dh)
            y0, y1, z = _project32(m, t, x, y, d)
            u32 = (y0 / z).astype(np.float64)
            v32 = (y1 / z).astype(np.float64)
            u64, v64, z64 = _project64(c2w[f], c2w[j], x, y, d, fx, fy, cx, cy)
            ok = (z64 > 0.5) & (np.abs(u64) < 3 * wl.spec.width) & (np.abs(v64) < 3 * wl.spec.height)
            du = np.maximum(np.abs(u32 - u64), np.abs(v32 - v64))
            max_du = max(max_du, float(du[ok].max()))
    print(f"depth estimate: max |du| {max_du:.3g} px (band {odepth.RND_BAND:.3g})")
    assert max_du <= odepth.RND_BAND / 5
