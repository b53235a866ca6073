"""Pins of the depth-agnostic frustum gather oracle (Sec. 4, Eq. 1-2): hand-derived
member sets for simple camera motions, the depth range, rho, and agreement with the
paper's own hull-rasterisation algorithm on random tiny scenes."""
import numpy as np
import pytest

from oracle import frustum as ofr
from oracle.gather import ID_SHIFT

FX = 100.0


def _translated(tx=0.0, ty=0.0, tz=0.0):
    c = np.eye(4)
    c[:3, 3] = (tx, ty, tz)
    return c


def _members(sets, i):
    return [int(v) for v in sets.ids[sets.offsets[i]:sets.offsets[i + 1]]]


def _q(ids):
    """(J - f + w, q) of each id"""
    return [(v >> ID_SHIFT, v & ((1 << ID_SHIFT) - 1)) for v in ids]


def test_static_camera_gives_the_l1_cross_in_every_frame():
    # identical cameras: q comes back to itself, so |p - q|_1 < 3/2 is the cross of
    # p and its four neighbours (clipped at the border), whatever the depths
    n, h, w = 3, 6, 7
    rng = np.random.default_rng(1)
    depth = rng.uniform(1.0, 5.0, (n, h, w))
    cams = np.stack([np.eye(4)] * n)
    colour = rng.random((n, h, w, 3))
    s = ofr.gather_frustum(colour, depth, cams, FX, FX, 3.0, 2.5, 1, ofr.FrustumParams(window=1))
    p = 2 * w + 3
    want = sorted((jj << ID_SHIFT) | q for jj in range(3) for q in (p - w, p - 1, p, p + 1, p + w))
    assert _members(s, p) == want
    corner = 0
    assert _members(s, corner) == sorted((jj << ID_SHIFT) | q for jj in range(3) for q in (0, 1, w))
    assert not s.marginal.any()


def test_frustum_size_one_keeps_the_pixel_itself():
    n, h, w = 2, 5, 5
    depth = np.full((n, h, w), 2.0)
    cams = np.stack([np.eye(4)] * n)
    s = ofr.gather_frustum(np.zeros((n, h, w, 3)), depth, cams, FX, FX, 2.0, 2.0, 0,
                           ofr.FrustumParams(window=1, l=1.0))
    for p in range(h * w):
        assert _members(s, p) == [(1 << ID_SHIFT) | p, (2 << ID_SHIFT) | p]


def test_sideways_camera_shifts_the_cross():
    # camera 1 sits 0.015 right of camera 0; depth 2, fx 100: a pixel q of frame 1
    # lands at q + (0.75, 0) in frame 0. Members of p from frame 1: q = p - (dx, dy)
    # with |dx - 0.75| + |dy| < 1.5: (0, 0), (1, 0), (2, 0), (1, +-1)
    n, h, w = 2, 7, 9
    depth = np.full((n, h, w), 2.0)
    cams = np.stack([np.eye(4), _translated(tx=0.015)])
    s = ofr.gather_frustum(np.zeros((n, h, w, 3)), depth, cams, FX, FX, 4.0, 3.0, 0, ofr.FrustumParams(window=1))
    px, py = 5, 3
    p = py * w + px
    from_1 = [q for (jj, q) in _q(_members(s, p)) if jj == 2]
    want = sorted((py - dy) * w + (px - dx) for dx, dy in ((0, 0), (1, 0), (2, 0), (1, 1), (1, -1)))
    assert from_1 == want


def test_depth_range_and_rho():
    # a q whose point lies beyond `far` is not in V; one exactly at `far` is (bounds
    # included, flagged marginal); rho = (z' - d_p) / d_p
    n, h, w = 1, 5, 5
    depth = np.full((n, h, w), 2.0)
    depth[0, 2, 3] = 2000.0
    depth[0, 1, 2] = 1000.0
    depth[0, 3, 2] = 3.0
    cams = np.stack([np.eye(4)])
    colour = np.zeros((n, h, w, 3))
    s = ofr.gather_frustum(colour, depth, cams, FX, FX, 2.0, 2.0, 0, ofr.FrustumParams(window=0))
    p = 2 * w + 2
    got = [q for (_, q) in _q(_members(s, p))]
    assert got == [1 * w + 2, 2 * w + 1, 2 * w + 2, 3 * w + 2]   # (3, 2) at depth 2000 left out
    a, b = s.offsets[p], s.offsets[p + 1]
    rho = dict(zip(got, s.rho[a:b]))
    assert rho[2 * w + 2] == pytest.approx(0.0, abs=1e-15)
    assert rho[3 * w + 2] == pytest.approx(0.5, rel=1e-12)
    marg = dict(zip(got, s.marginal[a:b]))
    assert marg[1 * w + 2] and not marg[2 * w + 2]


def _rot(axis, deg):
    t = np.radians(deg)
    c, s = np.cos(t), np.sin(t)
    r = np.eye(4)
    i, j = [(1, 2), (0, 2), (0, 1)][axis]
    r[i, i], r[i, j], r[j, i], r[j, j] = c, -s, s, c
    return r


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_definition_equals_the_papers_hull_rasterisation(seed):
    # random depths; the output camera at the origin, the others sideways and at
    # least 2 cm behind it, turned a little, so every frustum (whose near face is
    # 1 cm in front of the output camera) stays in front of every camera
    rng = np.random.default_rng(seed)
    n, h, w = 4, 10, 12
    depth = rng.uniform(1.0, 4.0, (n, h, w))
    depth[rng.random((n, h, w)) < 0.05] = np.nan
    f = 1
    cams = []
    for j in range(n):
        c = _translated(*rng.uniform(-0.08, 0.08, 2), tz=-rng.uniform(0.02, 0.15))
        c = c @ _rot(0, rng.uniform(-2, 2)) @ _rot(1, rng.uniform(-2, 2)) @ _rot(2, rng.uniform(-5, 5))
        cams.append(np.eye(4) if j == f else c)
    cams = np.stack(cams)
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    prm = ofr.FrustumParams(window=2)
    s = ofr.gather_frustum(rng.random((n, h, w, 3)), depth, cams, FX, FX, cx, cy, f, prm)
    seg = np.repeat(np.arange(h * w), np.diff(s.offsets))
    unsure = s.near_miss.copy()
    unsure[seg[s.marginal]] = True
    total = 0
    for p in range(h * w):
        if unsure[p]:
            continue
        hull = ofr.gather_frustum_hull(depth, cams, FX, FX, cx, cy, f, prm, p)
        assert _members(s, p) == hull, p
        total += len(hull)
    assert total > 2 * h * w   # the sets are not trivially empty
