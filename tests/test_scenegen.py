"""The seeded input generator: reproducible bit for bit, seed-dependent, and the
documented shapes, types and noise models."""
import torch

from scenegen import configs, generate


def _clip(seed):
    wl = configs.tiny(seed=seed, width=40, height=30, n_frames=4, window=2)
    return wl, generate(wl.spec)


def test_same_seed_same_clip_bit_for_bit():
    _, a = _clip(3)
    _, b = _clip(3)
    for name in ("rgb_u8", "depth", "cam_to_world", "clean_u8", "depth_true", "poses_true", "face_id"):
        x, y = getattr(a, name), getattr(b, name)
        assert x.dtype == y.dtype and torch.equal(torch.nan_to_num(x.double(), 7.0), torch.nan_to_num(y.double(), 7.0)), name
    assert (a.fx, a.fy, a.cx, a.cy) == (b.fx, b.fy, b.cx, b.cy)


def test_other_seed_other_clip():
    _, a = _clip(3)
    _, b = _clip(4)
    assert not torch.equal(a.rgb_u8, b.rgb_u8)
    assert not torch.equal(a.cam_to_world, b.cam_to_world)


def test_shapes_types_and_noise_models():
    wl, c = _clip(5)
    n, h, w = 4, 30, 40
    assert c.rgb_u8.shape == (n, h, w, 3) and c.rgb_u8.dtype == torch.uint8
    assert c.depth.shape == (n, h, w) and c.depth.dtype == torch.float32
    assert c.cam_to_world.shape == (n, 4, 4) and c.cam_to_world.dtype == torch.float64
    assert c.clean.shape == (n, h, w, 3) and float(c.clean.min()) >= 0.0 and float(c.clean.max()) <= 1.0
    # camera matrices are rigid: orthonormal rotation, last row (0, 0, 0, 1)
    r = c.cam_to_world[:, :3, :3]
    eye = torch.eye(3, dtype=torch.float64).expand(n, 3, 3)
    assert torch.allclose(r @ r.transpose(1, 2), eye, atol=1e-12)
    assert torch.equal(c.cam_to_world[:, 3], torch.tensor([0.0, 0.0, 0.0, 1.0], dtype=torch.float64).expand(n, 4))
    # the observed colour is the clean radiance plus noise: not equal, but close on average
    diff = (c.rgb_u8.double() - c.clean_u8.double()) / 255.0
    assert 0.5 * wl.spec.colour_sigma < float(diff.std()) < 2.0 * wl.spec.colour_sigma
    # depth outliers: replaced values far from the true depth, at about the configured rate
    rel = ((c.depth - c.depth_true).abs() / c.depth_true)
    outl = float((rel > 0.5).double().mean())
    assert outl < 4 * wl.spec.outlier_frac + 0.01
