"""Pins of the oracle's deblurring, shutter and inpainting filters (Sec. 5,
Eq. 5, Eq. 8-10) against closed forms and values worked out by hand."""
import math

import numpy as np
import pytest

from oracle import filters as of
from oracle.gather import ID_SHIFT, OracleSets


def _sets(frame, window, members, h=4, w=4):
    """OracleSets for output pixels 0, 1, ... of `frame`; members[i] = list of
    (source frame J, source pixel q, (r, g, b), rho)."""
    offsets, ids, colour, rho = [0], [], [], []
    for mem in members:
        for (j, q, c, r) in mem:
            ids.append(((j - frame + window) << ID_SHIFT) | q)
            colour.append(c)
            rho.append(r)
        offsets.append(len(ids))
    n = len(members)
    z = np.zeros(n + 1, dtype=np.int64)
    return OracleSets(frame=frame, pixels=np.arange(n, dtype=np.int64), offsets=np.array(offsets, dtype=np.int64),
                      ids=np.array(ids, dtype=np.uint32), rho=np.array(rho, dtype=np.float64),
                      colour=np.array(colour, dtype=np.float64).reshape(-1, 3),
                      marginal=np.zeros(len(ids), dtype=bool), maybe_offsets=z,
                      maybe_ids=np.zeros(0, dtype=np.uint32), maybe_rho=np.zeros(0))


def _colour_f(h=4, w=4, value=0.5):
    return np.full((h, w, 3), value)


# ---------------------------------------------------------------------------
# B(J), Eq. 5

def test_sharpness_of_constant_frames_is_zero():
    c = np.full((3, 5, 7, 3), 0.3)
    assert np.array_equal(of.frame_sharpness(c), np.zeros(3))


def test_sharpness_of_a_ramp():
    # I_c(x, y) = a_c x + b_c y: every counted pixel has |grad| = sqrt(sum a_c^2 + b_c^2);
    # (W - 1)(H - 1) pixels are counted
    h, w = 6, 9
    a, b = np.array([0.01, 0.02, -0.03]), np.array([0.005, 0.0, 0.04])
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    c = xx[..., None] * a + yy[..., None] * b
    want = (w - 1) * (h - 1) * math.sqrt(float(np.sum(a * a + b * b)))
    assert of.frame_sharpness(c[None])[0] == pytest.approx(want, rel=1e-12)


def test_sharpness_of_an_impulse():
    # value 1 at interior (x0, y0) in one channel: (x0, y0) has gx = gy = -1 (sqrt 2),
    # its left neighbour gx = +1 (1), its upper neighbour gy = +1 (1): 2 + sqrt 2
    c = np.zeros((2, 5, 6, 3))
    c[1, 2, 3, 1] = 1.0
    got = of.frame_sharpness(c)
    assert got[0] == 0.0
    assert got[1] == pytest.approx(2.0 + math.sqrt(2.0), rel=1e-15)


def test_sharpness_on_the_last_row_and_column_is_not_counted():
    # an impulse in the last column is seen only by its left neighbour (gx = +1)
    c = np.zeros((1, 4, 5, 3))
    c[0, 1, 4, 0] = 1.0
    assert of.frame_sharpness(c)[0] == pytest.approx(1.0, rel=1e-15)


def test_blurring_a_frame_lowers_its_sharpness():
    rng = np.random.default_rng(0)
    c = rng.random((1, 32, 32, 3))
    k = np.ones(3) / 3.0
    blurred = np.apply_along_axis(lambda v: np.convolve(v, k, mode="same"), 2, c)
    blurred = np.apply_along_axis(lambda v: np.convolve(v, k, mode="same"), 1, blurred)
    assert of.frame_sharpness(blurred)[0] < 0.5 * of.frame_sharpness(c)[0]


# ---------------------------------------------------------------------------
# per-frame factors, Eq. 5 / Eq. 10

def test_shutter_box_is_the_mean_over_its_frames():
    # sigma all +inf: w = xi(J); frames 3, 4, 5 with factors 1, 2, 0
    f, win = 4, 2
    sets = _sets(f, win, [[(3, 0, (0.1, 0.2, 0.3), 0.0), (4, 1, (0.4, 0.5, 0.6), 0.0),
                           (5, 2, (0.7, 0.8, 0.9), 0.0), (4, 3, (0.2, 0.2, 0.2), 0.0)]])
    xi = np.zeros(8)
    xi[3], xi[4], xi[5] = 1.0, 2.0, 0.0
    got = of.frame_weighted_mean(sets, _colour_f(), win, xi, math.inf)
    # (1 * (.1, .2, .3) + 2 * (.4, .5, .6) + 2 * (.2, .2, .2)) / 5
    np.testing.assert_allclose(got[0], [1.3 / 5, 1.6 / 5, 1.9 / 5], rtol=1e-14)


def test_frame_factor_times_depth_gaussian():
    # rho = 0.1 with sigma_d = 0.1: factor e^-1/2; rho = 0: factor 1; frame factors 3 and 1
    f, win = 2, 1
    sets = _sets(f, win, [[(1, 0, (1.0, 0.0, 0.0), 0.1), (2, 5, (0.0, 1.0, 0.0), 0.0)]])
    fw = np.array([0.0, 3.0, 1.0, 0.0])
    got = of.frame_weighted_mean(sets, _colour_f(), win, fw, 0.1)
    wa, wb = 3.0 * math.exp(-0.5), 1.0
    np.testing.assert_allclose(got[0], [wa / (wa + wb), wb / (wa + wb), 0.0], rtol=1e-14, atol=1e-300)


def test_frame_factors_are_scale_free_and_ones_give_the_plain_filter():
    rng = np.random.default_rng(3)
    f, win = 3, 3
    members = [[(int(rng.integers(0, 7)), int(rng.integers(0, 16)), tuple(rng.random(3)), float(rng.normal(0, 0.01)))
                for _ in range(int(rng.integers(1, 9)))] for _ in range(6)]
    sets = _sets(f, win, members)
    cf = rng.random((4, 4, 3))
    fw = rng.random(7) + 0.1
    a = of.frame_weighted_mean(sets, cf, win, fw, 0.01, 0.2, 2.0)
    b = of.frame_weighted_mean(sets, cf, win, 7.5 * fw, 0.01, 0.2, 2.0)
    np.testing.assert_allclose(a, b, rtol=1e-13)
    ones = of.frame_weighted_mean(sets, cf, win, np.ones(7), 0.01, 0.2, 2.0)
    np.testing.assert_allclose(ones, of.weighted_mean(sets.offsets, sets.colour, sets.rho,
                                                      (sets.ids.astype(np.int64) >> ID_SHIFT) - win,
                                                      cf.reshape(-1, 3)[sets.pixels], 0.01, 0.2, 2.0), rtol=1e-13)


def test_zero_factors_and_empty_sets_return_the_input_colour():
    f, win = 1, 1
    sets = _sets(f, win, [[(0, 1, (0.9, 0.9, 0.9), 0.0), (2, 1, (0.8, 0.8, 0.8), 0.0)], []])
    cf = np.zeros((4, 4, 3))
    cf[0, 0] = (0.1, 0.2, 0.3)
    cf[0, 1] = (0.4, 0.5, 0.6)
    got = of.frame_weighted_mean(sets, cf, win, np.array([0.0, 5.0, 0.0]), math.inf)
    np.testing.assert_array_equal(got, [[0.1, 0.2, 0.3], [0.4, 0.5, 0.6]])


# ---------------------------------------------------------------------------
# inpainting, Eq. 8-9

def _mask(frames=3, h=4, w=4, on=()):
    m = np.zeros((frames, h, w), dtype=bool)
    for (j, q) in on:
        m[j].reshape(-1)[q] = True
    return m


def test_inpaint_two_steps_follow_the_logistic_closed_form():
    # unmasked a = 0 and b = 1 (red channel), masked x = 1.25: s0 = 0.75. With two
    # samples, s_new = w_b / (w_a + w_b) = 1 / (1 + exp(-(2 s - 1) / (2 sigma^2)))
    f, win, sigma = 1, 1, 0.5
    g = 0.5
    sets = _sets(f, win, [[(0, 2, (0.0, g, g), 0.0), (2, 3, (1.0, g, g), 0.0), (0, 7, (1.25, g, g), 0.0)]])
    mask = _mask(on=[(1, 0), (0, 7)])
    got = of.inpaint_mean_shift(sets, _colour_f(value=0.2), win, mask, sigma, steps=2)
    s = 0.75
    for _ in range(2):
        s = 1.0 / (1.0 + math.exp(-(2.0 * s - 1.0) / (2.0 * sigma * sigma)))
    np.testing.assert_allclose(got[0], [s, g, g], rtol=1e-14)
    assert abs(s - 0.7159) < 1e-3


def test_inpaint_with_infinite_sigma_is_the_mean_of_unmasked_samples():
    f, win = 1, 1
    cols = [(0.1, 0.2, 0.3), (0.5, 0.1, 0.9), (0.9, 0.9, 0.0), (0.3, 0.3, 0.3)]
    sets = _sets(f, win, [[(0, 1, cols[0], 0.0), (1, 2, cols[1], 0.0), (2, 3, cols[2], 0.0), (2, 4, cols[3], 0.0)]])
    mask = _mask(on=[(1, 0), (2, 3)])   # output pixel 0 masked; sample (2, 3) masked
    got = of.inpaint_mean_shift(sets, _colour_f(), win, mask, 1e300, steps=2)
    want = (np.array(cols[0]) + np.array(cols[1]) + np.array(cols[3])) / 3.0
    np.testing.assert_allclose(got[0], want, rtol=1e-14)


def test_inpaint_follows_the_majority_cluster():
    # three unmasked samples near 0.2, one at 0.9: the mean-shift moves from the
    # overall mean (0.375) to the cluster of three
    f, win = 1, 1
    mem = [(0, 1, (0.19, 0.2, 0.2), 0.0), (0, 2, (0.2, 0.2, 0.2), 0.0), (2, 3, (0.21, 0.2, 0.2), 0.0),
           (2, 4, (0.9, 0.2, 0.2), 0.0)]
    got = of.inpaint_mean_shift(_sets(f, win, [mem]), _colour_f(), win, _mask(on=[(1, 0)]), 0.1, steps=2)
    assert abs(got[0, 0] - 0.2) < 0.01


def test_inpaint_leaves_unmasked_all_masked_and_empty_pixels():
    f, win = 1, 1
    cf = np.zeros((4, 4, 3))
    cf.reshape(-1, 3)[:3] = [(0.1, 0.1, 0.1), (0.2, 0.2, 0.2), (0.3, 0.3, 0.3)]
    sets = _sets(f, win, [[(0, 1, (0.9, 0.9, 0.9), 0.0)],      # pixel 0: not masked
                          [(0, 5, (0.9, 0.9, 0.9), 0.0)],      # pixel 1: masked, only a masked sample
                          []])                                 # pixel 2: masked, empty set
    mask = _mask(on=[(1, 1), (1, 2), (0, 5)])
    got = of.inpaint_mean_shift(sets, cf, win, mask, 0.2)
    np.testing.assert_array_equal(got, cf.reshape(-1, 3)[:3])


# ---------------------------------------------------------------------------
# masks from a scene-space box

def _cams(*mats):
    return np.stack([np.asarray(m, dtype=np.float64) for m in mats])


def test_box_mask_of_a_fronto_parallel_plane_is_a_rectangle():
    # identity camera, depth 2, f = 100, c = (10, 8): X = 2 (x - 10) / 100, Y = 2 (y - 8) / 100.
    # |X| <= 0.1 <=> 5 <= x <= 15; -0.04 <= Y <= 0.06 <=> 6 <= y <= 11
    h, w = 20, 24
    d = np.full((1, h, w), 2.0)
    m = of.scene_box_mask(d, _cams(np.eye(4)), 100.0, 100.0, 10.0, 8.0, (-0.1, -0.04, 1.0), (0.1, 0.06, 3.0))
    want = np.zeros((h, w), dtype=bool)
    want[6:12, 5:16] = True
    assert np.array_equal(m[0], want)


def test_box_mask_follows_the_camera_pose():
    # camera 1 translated by +0.2 along world X, camera 2 rotated 90 degrees about Z
    # (camera x -> world y): the same world box selects shifted / transposed pixels
    h, w = 20, 24
    d = np.full((3, h, w), 2.0)
    t = np.eye(4)
    t[0, 3] = 0.2
    rz = np.array([[0.0, -1.0, 0.0, 0.0], [1.0, 0.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
    lo, hi = (-0.1, -0.04, 1.0), (0.1, 0.06, 3.0)
    m = of.scene_box_mask(d, _cams(np.eye(4), t, rz), 100.0, 100.0, 10.0, 8.0, lo, hi)
    # frame 1: X = 2 (x - 10) / 100 + 0.2 in [-0.1, 0.1] <=> -5 <= x <= 5
    want1 = np.zeros((h, w), dtype=bool)
    want1[6:12, 0:6] = True
    assert np.array_equal(m[1], want1)
    # frame 2: world X = -Yc = -2 (y - 8) / 100 in [-0.1, 0.1] <=> 3 <= y <= 13;
    # world Y = Xc = 2 (x - 10) / 100 in [-0.04, 0.06] <=> 8 <= x <= 13
    want2 = np.zeros((h, w), dtype=bool)
    want2[3:14, 8:14] = True
    assert np.array_equal(m[2], want2)


def test_box_mask_depth_range_and_invalid_depths():
    h, w = 6, 6
    d = np.full((1, h, w), 2.0)
    d[0, 0, 0] = np.nan
    d[0, 0, 1] = np.inf
    d[0, 0, 2] = 0.0
    d[0, 1, :] = 5.0                       # behind the box's far face
    m = of.scene_box_mask(d, _cams(np.eye(4)), 1e6, 1e6, 2.5, 2.5, (-1.0, -1.0, 1.5), (1.0, 1.0, 2.0))
    want = np.ones((h, w), dtype=bool)
    want[0, :3] = False
    want[1, :] = False
    assert np.array_equal(m[0], want)      # z = 2.0 on the far face is inside (bounds included)


# ---------------------------------------------------------------------------
# Eq. 4 with the scene-space term, and semi-transparency

def _two_cameras():
    """Frame 0 at the origin, frame 1 translated by (0.5, 0, 0), no rotation;
    fx = fy = 100, cx = cy = 0; 4 x 4 images (only the listed pixels matter)."""
    cams = np.stack([np.eye(4), np.eye(4)])
    cams[1, 0, 3] = 0.5
    return cams


def test_scene_space_distances_worked_by_hand():
    """Frame 0 at the origin, frame 1 translated by (0.5, 0, 0); fx = fy = 100,
    (cx, cy) = (40, 1); images 64 x 4. Output pixel p = (40, 1) of frame 0 with depth
    2: X_ref = (0, 0, 2). Samples: p itself (distance 0); frame 1 pixel (15, 1) at
    depth 2: X = (2 (-25) / 100 + 0.5, 0, 2) = X_ref (distance 0); frame 1 pixel
    (20, 1) at depth 2: X = (0.1, 0, 2) (distance^2 0.01); frame 1 pixel (15, 2) at
    depth 2.2: X = (-0.55 + 0.5, 0.022, 2.2) (distance^2 0.0025 + 0.022^2 + 0.04).
    With sigma_xyz = 0.1 the weights are 1, 1, e^-0.5 and e^-(0.042984 / 0.02)."""
    w_img, h_img, cx, cy = 64, 4, 40.0, 1.0
    cams = _two_cameras()
    depth = np.full((2, h_img, w_img), 5.0)
    depth[0, 1, 40] = 2.0
    depth[1, 1, 15] = 2.0
    depth[1, 1, 20] = 2.0
    depth[1, 2, 15] = 2.2
    cols = [(0.1, 0.2, 0.3), (0.4, 0.5, 0.6), (0.9, 0.1, 0.5), (0.2, 0.8, 0.7)]
    p = w_img + 40
    sets = _sets(0, 1, [[(0, p, cols[0], 0.0), (1, w_img + 15, cols[1], 0.0), (1, w_img + 20, cols[2], 0.0),
                         (1, 2 * w_img + 15, cols[3], 0.0)]], h=h_img, w=w_img)
    sets.pixels = np.array([p], dtype=np.int64)
    colour_f = np.zeros((h_img, w_img, 3))
    colour_f[1, 40] = cols[0]
    got = of.scene_space_weighted_mean(sets, colour_f, depth, cams, 100.0, 100.0, cx, cy, 1,
                                       math.inf, math.inf, 0.1, math.inf)
    wts = np.array([1.0, 1.0, math.exp(-0.5), math.exp(-0.042984 / 0.02)])
    want = (wts[:, None] * np.array(cols)).sum(0) / wts.sum()
    assert np.allclose(got[0], want, rtol=0, atol=1e-14)
    # sigma_xyz infinite: the plain mean; the frame factor multiplies each weight
    got = of.scene_space_weighted_mean(sets, colour_f, depth, cams, 100.0, 100.0, cx, cy, 1,
                                       math.inf, math.inf, math.inf, math.inf)
    assert np.allclose(got[0], np.mean(cols, axis=0), atol=1e-15)
    got = of.scene_space_weighted_mean(sets, colour_f, depth, cams, 100.0, 100.0, cx, cy, 1,
                                       math.inf, math.inf, 0.1, math.inf, frame_w=np.array([3.0, 0.0]))
    assert np.allclose(got[0], cols[0], atol=1e-15)
    # an output pixel without a valid depth has no reference point: I^f(p)
    depth[0, 1, 40] = np.nan
    got = of.scene_space_weighted_mean(sets, colour_f, depth, cams, 100.0, 100.0, cx, cy, 1,
                                       math.inf, math.inf, 0.1, math.inf)
    assert np.array_equal(got[0], np.array(cols[0]))


def test_scene_space_term_is_invariant_to_a_rigid_motion_of_the_world():
    """Moving every camera by the same rigid transform moves every scene point with
    it, so no distance (and no output) changes."""
    rng = np.random.default_rng(3)
    w_img, h_img = 12, 9
    depth = 2.0 + 3.0 * rng.random((3, h_img, w_img))
    cams = np.stack([np.eye(4)] * 3)
    for j in range(3):
        a = rng.normal(size=3) * 0.05
        cams[j, :3, :3] = _rot(a)
        cams[j, :3, 3] = rng.normal(size=3) * 0.2
    g = np.eye(4)
    g[:3, :3] = _rot(np.array([0.3, -0.7, 1.1]))
    g[:3, 3] = [4.0, -2.0, 9.0]
    members = []
    for i in range(6):
        members.append([(j, int(rng.integers(0, w_img * h_img)), tuple(rng.random(3)), 0.0)
                        for j in (0, 1, 2) for _ in range(3)])
    sets = _sets(1, 1, members, h=h_img, w=w_img)
    sets.pixels = rng.choice(w_img * h_img, 6, replace=False).astype(np.int64)
    colour_f = rng.random((h_img, w_img, 3))
    args = (30.0, 30.0, 5.5, 4.0, 1, math.inf, 0.2, 0.3, 1.5)
    a = of.scene_space_weighted_mean(sets, colour_f, depth, cams, *args)
    b = of.scene_space_weighted_mean(sets, colour_f, depth, g @ cams, *args)
    assert np.allclose(a, b, rtol=0, atol=1e-12)
    assert not np.allclose(a, of.scene_space_weighted_mean(sets, colour_f, depth, cams, 30.0, 30.0, 5.5, 4.0, 1,
                                                           math.inf, 0.2, math.inf, 1.5), atol=1e-6)


def _rot(v):
    th = float(np.linalg.norm(v))
    k = v / th
    kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * kx + (1 - math.cos(th)) * (kx @ kx)


def test_semi_transparency_two_sample_closed_form():
    """Masked output pixel with input colour I = c1 and two unmasked samples c1, c2:
    the first step starts from the mean (c1 + c2) / 2, equidistant from both, so the
    inpainting factors are equal and only the factor around the input remains:
    s_1 = (c1 + e^-b c2) / (1 + e^-b), b = |c2 - c1|^2 / (2 sigma_ref^2). With
    sigma_ref infinite it is plain inpainting, (c1 + c2) / 2 after one step."""
    c1, c2 = np.array([0.2, 0.3, 0.4]), np.array([0.6, 0.3, 0.1])
    sets = _sets(0, 0, [[(0, 5, tuple(c1), 0.0), (0, 6, tuple(c2), 0.0)]])
    colour_f = np.zeros((4, 4, 3))
    colour_f[0, 0] = c1
    mask = np.zeros((1, 4, 4), bool)
    mask[0, 0, 0] = True
    sr = 0.3
    b = float(np.sum((c2 - c1) ** 2)) / (2 * sr * sr)
    got = of.inpaint_mean_shift(sets, colour_f, 0, mask, 0.2, steps=1, sigma_ref=sr)
    assert np.allclose(got[0], (c1 + math.exp(-b) * c2) / (1 + math.exp(-b)), atol=1e-15)
    got = of.inpaint_mean_shift(sets, colour_f, 0, mask, 0.2, steps=1)
    assert np.allclose(got[0], (c1 + c2) / 2, atol=1e-15)
