"""GPU parity of the data-term-only depth estimate (Sec. 3, preprocessing) through
the C ABI against the float64 oracle; all inputs seeded and synthetic."""
import numpy as np
import pytest
import torch

from oracle import depth as odepth
from oracle import staging as ostaging
from scenegen import configs, generate

pytestmark = pytest.mark.gpu

FX = 100.0


def _sg():
    import paper_2102_03011_amd as sg
    return sg


def _translated(tx):
    c = np.eye(4)
    c[0, 3] = tx
    return c


def test_textured_plane_depth_is_exact():
    # frames 1 and 2 moved by +-0.04 along x, a plane at depth 2: disparity 2 px
    # (I^1(x) = I^0(x + 2), I^2(x) = I^0(x - 2)); every wrong hypothesis lands a pixel
    # or more away in some counted frame, so the interior recovers 2 exactly
    sg = _sg()
    h, w, s = 20, 40, 2
    rng = np.random.default_rng(0)
    tex = rng.integers(0, 256, (h, w + 2 * s, 3), dtype=np.uint8)
    rgb = np.stack([tex[:, s:s + w], tex[:, 2 * s:2 * s + w], tex[:, 0:w]])
    cams = np.stack([np.eye(4), _translated(0.04), _translated(-0.04)])
    staged = sg.scene_stage(torch.from_numpy(np.ascontiguousarray(rgb)).cuda(),
                            torch.full((3, h, w), 2.0, dtype=torch.float32, device="cuda"),
                            torch.from_numpy(cams).cuda(), FX, FX, (w - 1) / 2, (h - 1) / 2)
    hyp = torch.tensor([1.0, 4.0 / 3.0, 2.0, 4.0, 8.0], dtype=torch.float32, device="cuda")
    d, cost = sg.scene_estimate_depth(staged, 0, 2, hyp)
    d, cost = d.cpu().numpy(), cost.cpu().numpy()
    assert np.all(d[1:-1, 1:-1] == 2.0)
    assert np.all(cost[1:-1, 1:-1] == 0.0)
    assert np.isnan(d[0]).all() and np.isnan(d[:, 0]).all() and np.isinf(cost[-1]).all()


def test_depth_matches_oracle_outside_its_bands():
    # on a 48 x 32 image float32 carries a projection within ~1e-5 px of float64,
    # so the rounding band is taken 1e-4 px here
    sg = _sg()
    wl = configs.tiny(seed=6, width=48, height=32, n_frames=5, window=2)
    clip = generate(wl.spec)
    staged = sg.scene_stage(clip.rgb_u8.cuda().contiguous(), clip.depth.cuda().contiguous(),
                            clip.cam_to_world.cuda().contiguous(), clip.fx, clip.fy, clip.cx, clip.cy)
    f = 2
    true = clip.depth_true.numpy()
    lo, hi = 0.8 * float(np.nanmin(true)), 1.2 * float(np.nanmax(true))
    hyp = (1.0 / np.linspace(1.0 / lo, 1.0 / hi, 24)).astype(np.float32)
    d, cost = sg.scene_estimate_depth(staged, f, 2, torch.from_numpy(hyp).cuda())
    d, cost = d.cpu().numpy().astype(np.float64), cost.cpu().numpy().astype(np.float64)
    col = ostaging.colour_q(clip.rgb_u8.numpy())
    want, want_cost, band = odepth.estimate_depth(col, clip.cam_to_world.numpy(), clip.fx, clip.fy, clip.cx, clip.cy,
                                                  f, 2, hyp.astype(np.float64), with_bands=True, rnd_band=1e-4)
    assert band.mean() < 0.3
    ok = ~band
    both_nan = np.isnan(d) & np.isnan(want)
    assert np.all((d[ok] == want[ok]) | both_nan[ok])
    fin = ok & np.isfinite(want_cost)
    assert fin.sum() > 0.5 * d.size
    np.testing.assert_allclose(cost[fin], want_cost[fin], rtol=1e-4, atol=1e-7)
    assert np.all(np.isinf(cost[ok & ~np.isfinite(want_cost)]))
