"""Pins of the data-term depth oracle (Sec. 3, preprocessing): a textured plane
seen by sideways cameras at integer disparities, constant images, the patch cost."""
import numpy as np
import pytest

from oracle import depth as odepth

FX = 100.0


def _translated(tx):
    c = np.eye(4)
    c[0, 3] = tx
    return c


def test_textured_plane_depth_is_recovered_exactly():
    # frame 0 at the origin, frames 1 and 2 moved by +-0.04 along x; plane at depth 2:
    # disparity fx * t / z = 2 px, so I^1(x) = I^0(x + 2) and I^2(x) = I^0(x - 2)
    h, w, z0, s = 9, 14, 2.0, 2
    rng = np.random.default_rng(0)
    tex = rng.random((h, w + 2 * s, 3))
    frames = np.stack([tex[:, s:s + w], tex[:, 2 * s:2 * s + w], tex[:, 0:w]])
    t = s * z0 / FX
    cams = np.stack([np.eye(4), _translated(t), _translated(-t)])
    # disparities 4, 3, 2, 1, 0.5 px: every wrong hypothesis lands at least one pixel
    # away from the true one in some counted frame (nearest-pixel patches)
    hyp = np.array([1.0, 4.0 / 3.0, 2.0, 4.0, 8.0])
    d, cost = odepth.estimate_depth(frames, cams, FX, FX, (w - 1) / 2, (h - 1) / 2, 0, 2, hyp)
    inner = (slice(1, h - 1), slice(1, w - 1))
    assert np.all(d[inner] == z0)
    assert np.all(cost[inner] == 0.0)
    # the one-pixel border has no full patch in frame 0
    assert np.isnan(d[0]).all() and np.isnan(d[:, -1]).all()


def test_constant_images_take_the_first_hypothesis():
    h, w = 6, 7
    frames = np.full((3, h, w, 3), 0.4)
    cams = np.stack([np.eye(4), _translated(0.02), _translated(-0.02)])
    hyp = np.array([3.0, 1.0, 2.0])
    d, cost = odepth.estimate_depth(frames, cams, FX, FX, 3.0, 2.5, 1, 1, hyp)
    assert np.all(d[1:-1, 1:-2] == 3.0)
    assert np.all(cost[1:-1, 1:-2] == 0.0)
    # x = 5: every hypothesis projects its patch out of both other frames: no depth
    assert np.isnan(d[1:-1, -2]).all()


def test_patch_cost_is_the_sum_of_squared_rgb_differences():
    # same camera: the point comes back to p itself; I^J = I^f + 0.1 in every channel:
    # 9 pixels x 3 channels x 0.01 = 0.27
    h, w = 5, 5
    rng = np.random.default_rng(2)
    a = rng.random((h, w, 3))
    frames = np.stack([a, a + 0.1])
    cams = np.stack([np.eye(4), np.eye(4)])
    d, cost = odepth.estimate_depth(frames, cams, FX, FX, 2.0, 2.0, 0, 1, np.array([1.5]))
    assert cost[2, 2] == pytest.approx(0.27, rel=1e-12)
    assert d[2, 2] == 1.5


def test_a_pixel_list_gives_the_same_estimates():
    rng = np.random.default_rng(5)
    h, w = 8, 11
    frames = rng.random((3, h, w, 3))
    cams = np.stack([np.eye(4), _translated(0.03), _translated(-0.02)])
    hyp = np.array([1.0, 1.5, 2.5, 4.0])
    full = odepth.estimate_depth(frames, cams, FX, FX, 5.0, 3.5, 0, 2, hyp, with_bands=True)
    pix = np.array([0, 13, 27, 40, 52, 87])
    part = odepth.estimate_depth(frames, cams, FX, FX, 5.0, 3.5, 0, 2, hyp, with_bands=True, pixels=pix)
    for a, b in zip(full, part):
        np.testing.assert_array_equal(a.reshape(-1)[pix], b.reshape(-1)[pix])
    others = np.setdiff1d(np.arange(h * w), pix)
    assert np.isnan(part[0].reshape(-1)[others]).all()


def test_cost_intervals_collapse_to_the_costs_away_from_rounding_bands():
    """Without a band every interval is the exact mean cost of estimate_depth; with a
    band wider than half a pixel every projection may take both neighbours, so each
    interval contains the nominal cost."""
    rng = np.random.default_rng(4)
    h, w = 12, 16
    col = rng.random((3, h, w, 3))
    cams = np.stack([np.eye(4)] * 3)
    cams[0, 0, 3], cams[2, 0, 3] = -0.05, 0.07
    hyp = np.array([1.0, 1.7, 2.5, 4.0])
    pixels = np.arange(h * w)
    depth, best = odepth.estimate_depth(col, cams, 20.0, 20.0, 7.5, 5.5, 1, 1, hyp, pixels=pixels)
    lo, hi = odepth.cost_intervals(col, cams, 20.0, 20.0, 7.5, 5.5, 1, 1, hyp, pixels, rnd_band=0.0)
    fin = np.isfinite(lo)
    assert np.array_equal(lo[fin], hi[fin])
    got_best = np.where(fin, lo, np.inf).min(axis=1)
    ok = np.isfinite(best.reshape(-1))
    assert np.allclose(got_best[ok], best.reshape(-1)[ok], rtol=0, atol=1e-12)
    lo2, hi2 = odepth.cost_intervals(col, cams, 20.0, 20.0, 7.5, 5.5, 1, 1, hyp, pixels, rnd_band=0.6)
    both = fin & np.isfinite(hi2) & (hi2 > 0)
    assert both.any()
    assert np.all(lo2[both] <= lo[both] + 1e-12) and np.all(hi2[both] >= hi[both] - 1e-12)
