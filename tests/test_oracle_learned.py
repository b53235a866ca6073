"""Pins of the learned-weight oracle: bfloat16 rounding against torch's converter,
GELU identities, special cases that reduce to the plain filter, finite-difference
gradients, the first Adam step in closed form, and closed-form features on planar
scenes with exact poses."""
import math

import numpy as np
import pytest
import torch

from oracle import filters, gather, learned, poses


def test_bf16_round_matches_torch_converter():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 0.0, 65504.0, 1e-30]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(learned.bf16_round(x), want)
    assert learned.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0             # tie to even
    assert learned.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1.015625     # tie to even


def test_gelu_identities_and_derivative():
    z = np.linspace(-6, 6, 241)
    assert learned.gelu(np.array([0.0]))[0] == 0.0
    assert np.allclose(learned.gelu(z) - learned.gelu(-z), z, atol=1e-15)
    assert abs(learned.gelu(np.array([8.0]))[0] - 8.0) < 1e-12
    h = 1e-6
    fd = (learned.gelu(z + h) - learned.gelu(z - h)) / (2 * h)
    assert np.allclose(learned.gelu_grad(z), fd, atol=1e-8)
    # Phi(1) = 0.8413447460685429 (standard normal table)
    assert abs(learned.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def _random_sets(rng, sizes):
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    s = off[-1]
    return off, rng.random((s, 3)), rng.normal(size=(s, 8))


def test_zero_output_layer_is_arithmetic_mean():
    rng = np.random.default_rng(1)
    off, col, x = _random_sets(rng, [5, 1, 0, 17])
    mlp = learned.init_mlp(3)
    mlp.w3[:] = 0.0
    mlp.b3 = 0.0
    m, _ = learned.forward(learned.standardise(x, mlp), mlp)
    cref = rng.random((4, 3))
    o, a = learned.set_softmax_mean(m, col, off, cref)
    want = filters.weighted_mean(off, col, np.zeros(off[-1]), np.zeros(off[-1]), cref, math.inf)
    assert np.allclose(o, want, atol=1e-15)
    assert np.array_equal(o[2], cref[2])


def test_log_weight_logits_reproduce_the_plain_filter():
    rng = np.random.default_rng(2)
    off, col, _ = _random_sets(rng, [9, 30, 2])
    rho = rng.uniform(-0.01, 0.01, off[-1])
    cref = rng.random((3, 3))
    m = -rho ** 2 / (2 * 0.01 ** 2)           # ln w of the depth Gaussian
    o, a = learned.set_softmax_mean(m, col, off, cref)
    want = filters.weighted_mean(off, col, rho, np.zeros(off[-1]), cref, 0.01)
    assert np.allclose(o, want, atol=1e-14)
    for i in range(3):
        assert abs(a[off[i]:off[i + 1]].sum() - 1.0) < 1e-14


def test_set_output_is_permutation_invariant():
    rng = np.random.default_rng(3)
    off, col, x = _random_sets(rng, [12])
    mlp = learned.init_mlp(4)
    m, _ = learned.forward(x, mlp)
    o1, _ = learned.set_softmax_mean(m, col, off, np.zeros((1, 3)))
    perm = rng.permutation(12)
    o2, _ = learned.set_softmax_mean(m[perm], col[perm], off, np.zeros((1, 3)))
    assert np.allclose(o1, o2, atol=1e-15)
    assert np.array_equal(learned.lower_median(col, off), learned.lower_median(col[perm], off))


def test_backward_matches_central_differences():
    rng = np.random.default_rng(4)
    off, col, x = _random_sets(rng, [6, 9, 0, 4])
    mlp = learned.init_mlp(5)
    mlp.b1 = rng.normal(size=64) * 0.1
    mlp.b2 = rng.normal(size=64) * 0.1
    cref = rng.random((4, 3))
    clean = rng.random((4, 3))
    _, g, _ = learned.loss_and_grads(x, col, off, cref, clean, mlp)
    h = 1e-6
    for name, idx in [("w1", (3, 17)), ("b1", (5,)), ("w2", (40, 2)), ("b2", (63,)), ("w3", (11,)), ("b3", None)]:
        p = mlp.copy()
        q = mlp.copy()
        if idx is None:
            p.b3 += h
            q.b3 -= h
        else:
            getattr(p, name)[idx] += h
            getattr(q, name)[idx] -= h
        lp, _, _ = learned.loss_and_grads(x, col, off, cref, clean, p)
        lq, _, _ = learned.loss_and_grads(x, col, off, cref, clean, q)
        fd = (lp - lq) / (2 * h)
        got = g[name] if idx is None else g[name][idx]
        assert abs(got - fd) <= 1e-7 * max(1.0, abs(fd)) + 1e-10, (name, got, fd)


def test_first_adam_step_closed_form():
    mlp = learned.init_mlp(6)
    before = mlp.copy()
    g = {"w3": np.linspace(-1, 1, 64), "b3": 0.25}
    opt = learned.Adam(lr=0.01)
    opt.step(mlp, g)
    # first step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    want = before.w3 - 0.01 * g["w3"] / (np.abs(g["w3"]) + 1e-8)
    assert np.allclose(mlp.w3, want, atol=1e-15)
    assert abs(mlp.b3 - (before.b3 - 0.01 * 0.25 / (0.25 + 1e-8))) < 1e-15


def test_adam_three_steps_hand_computed():
    """Three steps on one scalar with gradients 1, -1, 2 (lr 0.1, beta1 0.9, beta2 0.999):
    worked by hand, m = 0.1, -0.01, 0.191 and v = 0.001, 0.001999, 0.005997001;
    bias-corrected m = 1, -0.01 / 0.19, 0.191 / 0.271 and v = 1, 1, 0.005997001 /
    0.002997001, so the parameter moves by -0.1, +0.05263157894736842 x 0.1 and
    -0.1 x 0.7047970479704797 / sqrt(2.001000667000111). From the second step on
    every moment decay and both bias corrections change the result."""
    mlp = learned.init_mlp(3)
    mlp.b3 = 0.0
    opt = learned.Adam(lr=0.1)
    want_theta = [-0.1, -0.1 + 0.005263157894736842, -0.1 + 0.005263157894736842 - 0.04982421404270304]
    want_m = [0.1, -0.01, 0.191]
    want_v = [0.001, 0.001999, 0.005997001]
    for t, g in enumerate([1.0, -1.0, 2.0]):
        opt.step(mlp, {"b3": g})
        assert abs(opt.m["b3"] - want_m[t]) < 1e-15
        assert abs(opt.v["b3"] - want_v[t]) < 1e-15
        # eps = 1e-8 moves each step by at most lr * 1e-8
        assert abs(mlp.b3 - want_theta[t]) < 1e-8 * (t + 1), (t, mlp.b3)


def test_adam_constant_gradient_moves_lr_every_step():
    """With a constant gradient c the bias-corrected moments are exactly c and c^2 at
    every step t, so each step moves the parameter by lr c / (|c| + eps); a bias
    correction that used the wrong power of beta would change the step from t = 2 on."""
    mlp = learned.init_mlp(4)
    before = mlp.w3.copy()
    c = np.linspace(-2.0, 2.0, 64)
    c[c == 0] = 0.5
    opt = learned.Adam(lr=0.01)
    for t in range(1, 21):
        opt.step(mlp, {"w3": c})
        assert np.allclose(mlp.w3, before - t * 0.01 * c / (np.abs(c) + 1e-8), atol=1e-12), t


def test_colour_median_feature_on_hand_built_sets():
    """Feature x2 = |c_s - lower median of the set|_2 on three hand-built sets of a
    single frame (ids with J = f): n = 4 (lower median = 2nd smallest per channel,
    (0.2, 0.5, 0.4)), n = 3 (the median, (0.5, 0.5, 0.9)) and n = 1 (0). Distances
    worked by hand: sqrt(0.26), sqrt(0.1), sqrt(0.18), sqrt(0.14); sqrt(0.32),
    sqrt(0.26), sqrt(0.74); 0."""
    w_img, h_img = 8, 4
    colour = np.array([[0.1, 0.5, 0.9], [0.3, 0.2, 0.4], [0.2, 0.8, 0.1], [0.4, 0.6, 0.7],
                       [0.9, 0.9, 0.9], [0.0, 0.5, 1.0], [0.5, 0.0, 0.2],
                       [0.7, 0.1, 0.3]])
    offsets = np.array([0, 4, 7, 8])
    pixels = np.array([9, 10, 20])
    pix_of = np.repeat(np.arange(3), np.diff(offsets))
    # every record is the output pixel itself, source frame f, window 1
    ids = ((1 << 22) | pixels[pix_of]).astype(np.uint32)
    depth = np.full((3, h_img, w_img), 5.0)
    cams = np.stack([np.eye(4)] * 3)
    feat = learned.features(pix_of, ids, np.zeros(8), colour, offsets, pixels, 1, depth, cams,
                            10.0, 10.0, 3.5, 1.5, window=1, radius=1)
    want = np.sqrt([0.26, 0.1, 0.18, 0.14, 0.32, 0.26, 0.74, 0.0])
    assert np.allclose(feat[:, 1], want, rtol=0, atol=1e-15)


def test_lower_median_brute_force():
    rng = np.random.default_rng(7)
    for n in range(1, 12):
        c = rng.integers(0, 5, size=(n, 3)).astype(float)
        off = np.array([0, n])
        got = learned.lower_median(c, off)[0]
        for ch in range(3):
            vals = sorted(c[:, ch])
            # lower median: at least half the values are <= it, and it is a member
            assert got[ch] == vals[(n - 1) // 2]
            assert sum(v <= got[ch] for v in vals) >= (n + 1) // 2


def _rot(axis, a):
    c, s = math.cos(a), math.sin(a)
    m = {0: [[1, 0, 0], [0, c, -s], [0, s, c]], 1: [[c, 0, s], [0, 1, 0], [-s, 0, c]],
         2: [[c, -s, 0], [s, c, 0], [0, 0, 1]]}[axis]
    return np.array(m, float)


def test_features_on_planar_scene_closed_forms():
    rng = np.random.default_rng(8)
    w_img, h_img, n_frames = 40, 30, 3
    fx = fy = 35.0
    cx, cy = (w_img - 1) / 2, (h_img - 1) / 2
    k = poses.intrinsics(fx, fy, cx, cy)
    cams = []
    for _ in range(n_frames):
        m = np.eye(4)
        m[:3, :3] = _rot(0, rng.normal() * 0.03) @ _rot(1, rng.normal() * 0.03)
        m[:3, 3] = rng.normal(size=3) * 0.1
        cams.append(m)
    cams = np.stack(cams)
    n_w = np.array([0.1, -0.3, -1.0])
    n_w /= np.linalg.norm(n_w)
    delta_w = -5.0

    def plane_depth(cam, xs, ys):
        r, t = cam[:3, :3], cam[:3, 3]
        n_c = r.T @ n_w
        d_c = delta_w - n_w @ t
        rays = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones_like(xs)], -1)
        return d_c / (rays @ n_c)

    ys, xs = np.mgrid[0:h_img, 0:w_img].astype(float)
    depth = np.stack([plane_depth(c, xs, ys) for c in cams])
    prm = gather.GatherParams(window=1, radius=1, tol=0.05)
    f = 1
    sets = gather.gather_frame(np.zeros(depth.shape + (3,)), depth, cams, fx, fy, cx, cy, f, prm)
    seg = np.repeat(np.arange(sets.pixels.size), np.diff(sets.offsets))
    feat = learned.features(seg, sets.ids, sets.rho, sets.colour, sets.offsets, sets.pixels, f, depth,
                            cams, fx, fy, cx, cy, window=1, radius=1)
    kinv = np.linalg.inv(k)
    dj = (sets.ids.astype(np.int64) >> 22) - 1
    q = sets.ids & ((1 << 22) - 1)
    checked = 0
    for s in range(0, sets.ids.size, 7):
        p = sets.pixels[seg[s]]
        x, y = p % w_img, p // w_img
        j = f + dj[s]
        qx, qy = q[s] % w_img, q[s] // w_img
        # world-frame point and camera centres
        dp = depth[f, y, x]
        xw = cams[f] @ np.append(dp * (kinv @ [x, y, 1.0]), 1.0)
        xj = np.linalg.solve(cams[j], xw)[:3]
        u, v = fx * xj[0] / xj[2] + cx, fy * xj[1] / xj[2] + cy
        assert abs(feat[s, 3] - math.hypot(qx - u, qy - v)) < 1e-9
        a, b = xw[:3] - cams[f][:3, 3], xw[:3] - cams[j][:3, 3]
        assert abs(feat[s, 4] - (1.0 - a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))) < 1e-12
        # depth gradient from the analytic plane depth at the neighbours
        def dd(xx, yy):
            return plane_depth(cams[j], np.array([float(xx)]), np.array([float(yy)]))[0]
        gx = 0.5 * (dd(qx + 1, qy) - dd(qx - 1, qy)) if 0 < qx < w_img - 1 else (
            dd(qx + 1, qy) - dd(qx, qy) if qx == 0 else dd(qx, qy) - dd(qx - 1, qy))
        gy = 0.5 * (dd(qx, qy + 1) - dd(qx, qy - 1)) if 0 < qy < h_img - 1 else (
            dd(qx, qy + 1) - dd(qx, qy) if qy == 0 else dd(qx, qy) - dd(qx, qy - 1))
        assert abs(feat[s, 5] - math.hypot(gx, gy) / dd(qx, qy)) < 1e-12
        assert feat[s, 2] == abs(dj[s]) and feat[s, 7] == dj[s]
        if dj[s] == 0 and qx == x and qy == y:
            assert feat[s, 0] == 0 and feat[s, 3] < 1e-12 and abs(feat[s, 4]) < 1e-15
        checked += 1
    assert checked > 300
    n = np.diff(sets.offsets)[seg]
    assert np.allclose(feat[:, 6], np.log1p(n) / math.log1p(27))
