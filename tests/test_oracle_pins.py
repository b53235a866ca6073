"""Pins of the float64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against a closed form, an invariant, an all-pairs
brute force, or numbers printed in the paper, so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import bruteforce, filters, gather, metrics, poses, staging
from scenegen import configs, generate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# helpers that build exact scenes (independent formulas, not oracle code)

def _rot(axis, ang):
    c, s = math.cos(ang), math.sin(ang)
    if axis == 0:
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == 1:
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def _random_rigid(rng, rot_scale=0.2, trans_scale=0.5):
    r = _rot(0, rng.normal() * rot_scale) @ _rot(1, rng.normal() * rot_scale) @ _rot(2, rng.normal() * rot_scale)
    m = np.eye(4)
    m[:3, :3] = r
    m[:3, 3] = rng.normal(size=3) * trans_scale
    return m


def _plane_depth(k, cam, n_w, delta_w, w, h):
    """Exact z-depth of the world plane n_w . X = delta_w seen by camera `cam` (camera-to-world)."""
    r, t = cam[:3, :3], cam[:3, 3]
    n_c = r.T @ n_w
    d_c = delta_w - n_w @ t
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    rays = np.stack([(xs - k[0, 2]) / k[0, 0], (ys - k[1, 2]) / k[1, 1], np.ones_like(xs)], -1)
    return d_c / (rays @ n_c)


# ----------------------------------------------------------------------------
# poses

def test_relative_pose_closed_form_and_invariants():
    rng = np.random.default_rng(3)
    cams = [_random_rigid(rng) for _ in range(4)]
    for a in range(4):
        assert np.array_equal(poses.relative(cams[a], cams[a], True), np.eye(4))
        for b in range(4):
            t = poses.relative(cams[a], cams[b], a == b)
            # closed form for rigid maps: (R_b^T R_a, R_b^T (t_a - t_b))
            ra, ta, rb, tb = cams[a][:3, :3], cams[a][:3, 3], cams[b][:3, :3], cams[b][:3, 3]
            assert np.allclose(t[:3, :3], rb.T @ ra, atol=1e-13)
            assert np.allclose(t[:3, 3], rb.T @ (ta - tb), atol=1e-13)
            back = poses.relative(cams[b], cams[a], a == b)
            assert np.allclose(t @ back, np.eye(4), atol=1e-13)
    loop = poses.relative(cams[2], cams[0], False) @ poses.relative(cams[1], cams[2], False) @ poses.relative(cams[0], cams[1], False)
    assert np.allclose(loop, np.eye(4), atol=1e-13)


# ----------------------------------------------------------------------------
# projection: planar scenes with exact poses and depths

def _planar_case(seed, w=48, h=32, n_frames=4):
    rng = np.random.default_rng(seed)
    fx = fy = 40.0
    cx, cy = (w - 1) / 2, (h - 1) / 2
    k = poses.intrinsics(fx, fy, cx, cy)
    cams = np.stack([_random_rigid(rng, 0.05, 0.15) for _ in range(n_frames)])
    n_w = np.array([0.25, -0.4, -1.0])
    n_w /= np.linalg.norm(n_w)
    delta_w = -6.0
    depth = np.stack([_plane_depth(k, cams[j], n_w, delta_w, w, h) for j in range(n_frames)])
    assert (depth > 2).all() and (depth < 20).all()
    return k, cams, n_w, delta_w, depth


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planar_homography_predicts_every_residual(seed):
    w, h = 48, 32
    k, cams, n_w, delta_w, depth = _planar_case(seed, w, h)
    colour = np.zeros(depth.shape + (3,))
    prm = gather.GatherParams(window=3, radius=1, tol=0.002)
    f = 1
    sets = gather.gather_frame(colour, depth, cams, k[0, 0], k[1, 1], k[0, 2], k[1, 2], f, prm)
    kinv = np.linalg.inv(k)
    rf, tf = cams[f][:3, :3], cams[f][:3, 3]
    n_f = rf.T @ n_w
    d_f = delta_w - n_w @ tf
    checked = 0
    for i, p in enumerate(sets.pixels):
        x, y = p % w, p // w
        pt = np.array([x, y, 1.0])
        got = {int(a): r for a, r in zip(sets.members_of(i), sets.rho[sets.offsets[i]:sets.offsets[i + 1]])}
        marg = set(int(a) for a, m in zip(sets.members_of(i), sets.marginal[sets.offsets[i]:sets.offsets[i + 1]]) if m)
        maybe = set(int(a) for a in sets.maybe_ids[sets.maybe_offsets[i]:sets.maybe_offsets[i + 1]])
        want = {}
        for j in range(0, 4):
            rj, tj = cams[j][:3, :3], cams[j][:3, 3]
            r_rel, t_rel = rj.T @ rf, rj.T @ (tf - tj)
            hmg = r_rel + np.outer(t_rel, n_f) / d_f            # plane-induced map X_f -> X_J
            pj = k @ hmg @ kinv @ pt
            u, v = pj[0] / pj[2], pj[1] / pj[2]
            dp = d_f / (n_f @ (kinv @ pt))
            z = (hmg @ (dp * (kinv @ pt)))[2]
            uh, vh = math.floor(u + 0.5), math.floor(v + 0.5)
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    qx, qy = uh + dx, vh + dy
                    if not (0 <= qx < w and 0 <= qy < h):
                        continue
                    rho = (depth[j, qy, qx] - z) / z
                    if abs(rho) <= 0.002:
                        want[((j - f + 3) << 22) | (qy * w + qx)] = rho
        for key, rho in want.items():
            if key in marg or key in maybe:
                continue
            assert key in got, (p, key)
            assert abs(got[key] - rho) < 1e-12
            checked += 1
        for key in got:
            assert key in want or key in marg, (p, key)
    assert checked > 1000


def test_fronto_parallel_plane_closed_form_count():
    # Every camera looks down the same axis at the plane z = 7 (rotation about the
    # optical axis only), so every source pixel lies on the plane: rho = 0 for all
    # candidates and the set size is the number of in-image block pixels.
    w, h, n_frames = 40, 30, 5
    fx = fy = 35.0
    cx, cy = (w - 1) / 2, (h - 1) / 2
    k = poses.intrinsics(fx, fy, cx, cy)
    rng = np.random.default_rng(11)
    cams = []
    for j in range(n_frames):
        m = np.eye(4)
        m[:3, :3] = _rot(2, rng.normal() * 0.05)
        m[:3, 3] = [rng.normal() * 0.3, rng.normal() * 0.3, rng.normal() * 0.5]
        cams.append(m)
    cams = np.stack(cams)
    depth = np.stack([np.full((h, w), 7.0 - cams[j][2, 3]) for j in range(n_frames)])
    prm = gather.GatherParams(window=n_frames, radius=1, tol=1e-9)
    f = 2
    sets = gather.gather_frame(np.zeros(depth.shape + (3,)), depth, cams, fx, fy, cx, cy, f, prm)
    kinv = np.linalg.inv(k)
    for i, p in enumerate(sets.pixels):
        x, y = p % w, p // w
        expect = 0
        for j in range(n_frames):
            # closed form: X on z = 7 - t_f,z; image of X in J is K R_z(theta) K^-1-like map
            rel = np.linalg.solve(cams[j], cams[f])
            xf = (7.0 - cams[f][2, 3]) * (kinv @ np.array([x, y, 1.0]))
            yj = rel[:3, :3] @ xf + rel[:3, 3]
            u, v = fx * yj[0] / yj[2] + cx, fy * yj[1] / yj[2] + cy
            uh, vh = math.floor(u + 0.5), math.floor(v + 0.5)
            if abs(u - math.floor(u) - 0.5) < 1e-6 or abs(v - math.floor(v) - 0.5) < 1e-6:
                expect = None
                break
            nx = sum(1 for d in (-1, 0, 1) if 0 <= uh + d < w)
            ny = sum(1 for d in (-1, 0, 1) if 0 <= vh + d < h)
            expect += nx * ny
        if expect is None:
            continue
        assert sets.offsets[i + 1] - sets.offsets[i] == expect
        assert np.all(np.abs(sets.rho[sets.offsets[i]:sets.offsets[i + 1]]) < 1e-12)


def test_zero_reprojection_error_on_plane():
    w, h = 48, 32
    k, cams, n_w, delta_w, depth = _planar_case(5, w, h)
    f, j = 0, 2
    ys, xs = np.mgrid[0:h, 0:w]
    x, y = xs.ravel().astype(float), ys.ravel().astype(float)
    t_rel = poses.relative(cams[f], cams[j], False)
    u, v, z = gather.project(depth[f].ravel(), x, y, t_rel, k)
    # back-project (u, v) with the plane depth in J and map into f
    rj = cams[j][:3, :3]
    n_j = rj.T @ n_w
    d_j = delta_w - n_w @ cams[j][:3, 3]
    rays = np.linalg.inv(k) @ np.stack([u, v, np.ones_like(u)])
    xj = rays * (d_j / (n_j @ rays))
    assert np.allclose(xj[2], z, rtol=1e-12)
    back = poses.relative(cams[j], cams[f], False)
    xf = back[:3, :3] @ xj + back[:3, 3:4]
    pf = k @ xf
    assert np.max(np.abs(pf[0] / pf[2] - x)) < 1e-9
    assert np.max(np.abs(pf[1] / pf[2] - y)) < 1e-9


# ----------------------------------------------------------------------------
# enumeration: all-pairs brute force on tiny random clips

@pytest.mark.parametrize("seed,window", [(0, 4), (1, 2), (2, 1)])
def test_bruteforce_all_pairs_equals_oracle(seed, window):
    wl = configs.tiny(seed=seed, pose_rot_deg=3.0, pose_trans_m=0.08, depth_noise=0.01, outlier_frac=0.05)
    clip = generate(wl.spec)
    dep = staging.depth_q(clip.depth.numpy())
    dep[1, 3, 4] = np.nan       # invalid depths must be skipped on both sides
    dep[2, 5, 7] = 0.0
    dep[0, 6, 6] = np.inf
    col = staging.colour_q(clip.rgb_u8.numpy())
    cams = clip.cam_to_world.numpy()
    prm = gather.GatherParams(window=window, radius=1, tol=0.01)
    total = 0
    for f in range(clip.n_frames):
        sets = gather.gather_frame(col, dep, cams, clip.fx, clip.fy, clip.cx, clip.cy, f, prm)
        bf = bruteforce.gather_all_pairs(dep, cams, clip.fx, clip.fy, clip.cx, clip.cy, f,
                                         window, 1, 0.01, 0.01)
        for i, p in enumerate(sets.pixels):
            mine = sets.members_of(i).tolist()
            marg = set(int(a) for a, m in zip(mine, sets.marginal[sets.offsets[i]:sets.offsets[i + 1]]) if m)
            maybe = set(sets.maybe_ids[sets.maybe_offsets[i]:sets.maybe_offsets[i + 1]].tolist())
            ref = [a for a, _ in bf[int(p)]]
            assert set(mine) - marg <= set(ref) <= set(mine) | maybe, (f, p)
            assert mine == sorted(mine)                      # canonical order
            rr = dict(bf[int(p)])
            for a, r in zip(mine, sets.rho[sets.offsets[i]:sets.offsets[i + 1]]):
                if a in rr:
                    assert abs(rr[a] - r) < 1e-12
            total += len(ref)
    assert total > 500


# ----------------------------------------------------------------------------
# end-to-end invariants with error-free data (Sec. 4: l = 1 holds every observation)

def test_static_camera_exact_data_returns_clean_frame():
    wl = configs.tiny(seed=4, width=24, height=16, n_frames=6, window=5, colour_sigma=0.0, depth_noise=0.0,
                      outlier_frac=0.0, pose_rot_deg=0.0, pose_trans_m=0.0, static_camera=True)
    clip = generate(wl.spec)
    col = staging.colour_q(clip.rgb_u8.numpy())
    dep = staging.depth_q(clip.depth.numpy())
    prm = gather.GatherParams(window=5, radius=0, tol=0.01)
    for f in (0, 3, 5):
        sets = gather.gather_frame(col, dep, clip.cam_to_world.numpy(), clip.fx, clip.fy, clip.cx, clip.cy, f, prm)
        # every frame of the window observes the same scene point exactly once
        assert np.all(np.diff(sets.offsets) == 6)
        out = filters.filter_sets(sets, col[f], 5, 0.01)
        assert np.abs(out - col[f].reshape(-1, 3)).max() < 1e-12
        assert np.array_equal(clip.rgb_u8[f].numpy(), clip.clean_u8[f].numpy())


def test_piecewise_constant_scene_interior_pixels_are_clean():
    wl = configs.tiny(seed=6, width=96, height=64, n_frames=7, window=3, colour_sigma=0.0, depth_noise=0.0,
                      outlier_frac=0.0, pose_rot_deg=0.0, pose_trans_m=0.0, piecewise_constant=True)
    wl.spec.n_static = 6
    clip = generate(wl.spec)
    col = staging.colour_q(clip.rgb_u8.numpy())
    dep = staging.depth_q(clip.depth.numpy())
    fid = clip.face_id.numpy()
    prm = gather.GatherParams(window=3, radius=1, tol=0.01)
    f = 3
    sets = gather.gather_frame(col, dep, clip.cam_to_world.numpy(), clip.fx, clip.fy, clip.cx, clip.cy, f, prm)
    out = filters.filter_sets(sets, col[f], 3, 0.01).reshape(col[f].shape)
    # interior: every pixel within 3 px (Chebyshev) has the same face id; what
    # lies beyond the image border is unknown and counts as a different face
    m = 3
    pad = np.pad(fid[f], m, mode="constant", constant_values=-1)
    interior = np.ones(fid[f].shape, bool)
    for dy in range(-m, m + 1):
        for dx in range(-m, m + 1):
            interior &= pad[m + dy:m + dy + fid.shape[1], m + dx:m + dx + fid.shape[2]] == fid[f]
    assert interior.sum() > 1000
    err = np.abs(out - col[f]).max(axis=-1)[interior]
    assert err.max() < 1e-12


# ----------------------------------------------------------------------------
# filter (Eq. 3 / Eq. 4) closed forms

def _csr(sizes):
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    return off


def test_filter_closed_forms():
    rng = np.random.default_rng(0)
    # set of size one returns its colour; equal colours return that colour
    off = _csr([1, 5])
    col = rng.random((6, 3))
    col[1:] = col[1]
    rho = rng.normal(size=6) * 0.01
    out = filters.weighted_mean(off, col, rho, np.zeros(6), rng.random((2, 3)), 0.01)
    assert np.allclose(out[0], col[0], atol=1e-15) and np.allclose(out[1], col[1], atol=1e-15)
    # infinite sigma: arithmetic mean (w = 1, the plain mean of the denoising section)
    off = _csr([7])
    col = rng.random((7, 3))
    out = filters.weighted_mean(off, col, rng.normal(size=7), np.arange(7), rng.random((1, 3)), math.inf)
    assert np.allclose(out[0], col.mean(0), atol=1e-15)
    # two samples with closed-form Gaussian weights on rho, colour distance and frame offset
    off = _csr([2])
    col = np.array([[0.2, 0.4, 0.6], [0.8, 0.1, 0.3]])
    cref = np.array([[0.25, 0.35, 0.6]])
    rho = np.array([0.004, -0.009])
    dj = np.array([0, -3])
    sd, sc, st = 0.01, 0.3, 6.0
    w0 = math.exp(-0.004 ** 2 / (2 * sd * sd)) * math.exp(-(0.05 ** 2 + 0.05 ** 2) / (2 * sc * sc))
    w1 = math.exp(-0.009 ** 2 / (2 * sd * sd)) * math.exp(-(0.55 ** 2 + 0.25 ** 2 + 0.3 ** 2) / (2 * sc * sc)) * math.exp(-9 / 72)
    want = (w0 * col[0] + w1 * col[1]) / (w0 + w1)
    out = filters.weighted_mean(off, col, rho, dj, cref, sd, sc, st)
    assert np.allclose(out[0], want, atol=1e-15)
    # empty set returns the reference colour
    out = filters.weighted_mean(_csr([0]), np.zeros((0, 3)), np.zeros(0), np.zeros(0), cref, 0.01)
    assert np.array_equal(out, cref)
    # sigma_d -> 0 keeps only rho = 0 samples ("at best recreate the original frame")
    off = _csr([3])
    col = rng.random((3, 3))
    out = filters.weighted_mean(off, col, np.array([0.0, 0.003, -0.004]), np.zeros(3), cref, 1e-5)
    assert np.allclose(out[0], col[0], atol=1e-12)


def test_filter_residual_variance_statistical():
    # flat colour, exact geometry, colour noise only: the residual of a weighted
    # mean of independent samples has variance sigma^2 * sum w^2 / (sum w)^2.
    rng = np.random.default_rng(1)
    n_sets, size, sigma = 20000, 40, 0.05
    off = _csr([size] * n_sets)
    rho = rng.uniform(-0.01, 0.01, size=n_sets * size)
    col = 0.5 + sigma * rng.normal(size=(n_sets * size, 3))
    out = filters.weighted_mean(off, col, rho, np.zeros(n_sets * size), np.full((n_sets, 3), 0.5), 0.01)
    w = np.exp(-rho ** 2 / (2 * 0.01 ** 2)).reshape(n_sets, size)
    var_pred = sigma ** 2 * (w ** 2).sum(1) / w.sum(1) ** 2
    z = (out - 0.5) ** 2 / var_pred[:, None]   # each term has mean 1, variance 2
    se = math.sqrt(2.0 / z.size)
    assert abs(z.mean() - 1.0) < 3 * se


# ----------------------------------------------------------------------------
# storage rounding and PSNR

def test_binary16_storage_known_encodings():
    assert staging.colour_q(np.array([255], np.uint8))[0] == 1.0
    assert staging.colour_q(np.array([128], np.uint8))[0] == 0.501953125     # 0x3804
    assert staging.colour_q(np.array([1], np.uint8))[0] == 0.0039215087890625  # 0x1C04
    d = staging.depth_q(np.array([65504.0, 65519.0, 65520.0, 3.0009765625, 3.0029296875], np.float32))
    assert d[0] == 65504 and d[1] == 65504 and np.isinf(d[2])
    assert d[3] == 3.0 and d[4] == 3.00390625   # ties go to even at spacing 2^-9


def test_psnr_closed_form_and_paper_noisy_input_column():
    golden = json.load(open(os.path.join(GOLDEN, "paper_denoise_psnr.json")))
    rng = np.random.default_rng(2)
    img = rng.uniform(0.3, 0.7, size=(256, 256, 3))
    for sigma, paper in zip(golden["sigma"], golden["noisy_input_psnr_db"]):
        noisy = img + rng.normal(size=img.shape) * sigma / 255.0
        got = metrics.psnr(noisy, img)
        closed = 20 * math.log10(255.0 / sigma)
        assert abs(got - closed) < 0.05
        if sigma <= 16:
            # the paper's measured noisy-input PSNR follows the same definition
            # (clipping of the real sequence only matters at large sigma)
            assert abs(paper - closed) < 0.3
    assert metrics.psnr(img, img) == float("inf")
