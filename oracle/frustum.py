"""Depth-agnostic frustum gather (Sec. 4, Eq. 1-2) -- test infrastructure only.

Output pixel p of frame f (camera C^f) defines the frustum V of Eq. 1: the
truncated pyramid over the square (p_x +- l/2, p_y +- l/2) between the depths
near and far (0.01 and 1000 in the paper). A pixel q of an input frame J with
stored depth D^J(q) is a member of S(p) when its scene point, carried into the
output view, lands within L1 distance l/2 of p (Eq. 2), strictly, and lies in
the frustum's depth range:

  X   = C^J [D^J(q) K^-1 (q_x, q_y, 1), 1]          (scene point of q)
  Y   = (C^f)^-1 X,  z' = Y_3,  p' = (fx Y_1 / z' + cx, fy Y_2 / z' + cy)
  q in S(p)  <=>  near <= z' <= far  and  |p_x - p'_x| + |p_y - p'_y| < l / 2.

The depth of p itself plays no part (the gather is depth-agnostic). This module
gives the plain definition (`gather_frustum`, every q of every window frame
against every output pixel it can reach) and, to pin it, the paper's own
algorithm (`gather_frustum_hull`: project the 8 corners of V into J, rasterise
their convex hull, apply Eq. 2 to the pixels inside). The two agree whenever V
lies in front of camera J, where the hull of the projected corners is the
projection of V. Reading: the frustum's depth range is part of membership (a
point behind the output camera or past `far` is not in V), bounds included.

Each sample also carries rho = (z' - d_p) / d_p, its relative depth offset along
p's ray from p's own scene point (reading: the scene-space distance to the
reference sample that Sec. 5 weights by, measured the way the depth-guided
path measures it); rho is NaN when p has no valid depth.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import poses as _poses
from .gather import ID_SHIFT

# Band flags for comparisons with a float32 evaluation of the same test: p' carried
# in float32 through float32-rounded pose maps is off by up to 7.0e-4 px (L1) at
# 1920x1080 with the full-scale workload's poses over a +-10 window, z' by up to
# 2.2e-7 relative (measured in tests/test_float32_bands.py); each band is at least
# five times that.
L1_BAND = 4e-3      # |L1 - l/2| below this (pixels): membership may differ in float32
Z_BAND = 1e-5       # relative distance of z' to near / far below this: likewise


@dataclass
class FrustumParams:
    window: int
    l: float = 3.0
    near: float = 0.01
    far: float = 1000.0


@dataclass
class FrustumSets:
    """S(p) for the listed output pixels of frame `frame`, CSR over the pixel list,
    members in ascending id ((J - f + w) << 22 | q)."""
    frame: int
    pixels: np.ndarray     # [n] flat y * W + x
    offsets: np.ndarray    # [n + 1] int64
    ids: np.ndarray        # [S] uint32
    rho: np.ndarray        # [S] float64
    colour: np.ndarray     # [S, 3] float64
    marginal: np.ndarray   # [S] bool: within a band of the L1 or depth-range bound
    near_miss: np.ndarray  # [n] bool: some non-member of p lies within such a band
    near_offsets: np.ndarray | None = None  # [n + 1] CSR over the pixel list: those non-members,
    near_ids: np.ndarray | None = None      # [M] ids, ascending per pixel


def carried_into_output(depth_j: np.ndarray, c_j: np.ndarray, c_f: np.ndarray, k: np.ndarray):
    """p' (x, y) and z' of every pixel q of frame J seen from output camera C^f."""
    h, w = depth_j.shape
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    kinv = np.linalg.inv(k)
    rays = kinv @ np.stack([xx.ravel(), yy.ravel(), np.ones(h * w)])            # [3, HW]
    with np.errstate(divide="ignore", invalid="ignore"):   # invalid depths give NaN points
        xcam = depth_j.ravel()[None, :] * rays
        xw = c_j[:3, :3] @ xcam + c_j[:3, 3:4]
        cf_inv = np.linalg.inv(c_f)
        yo = cf_inv[:3, :3] @ xw + cf_inv[:3, 3:4]
        z = yo[2]
        px = k[0, 0] * yo[0] / z + k[0, 2]
        py = k[1, 1] * yo[1] / z + k[1, 2]
    return px.reshape(h, w), py.reshape(h, w), z.reshape(h, w)


def gather_frustum(colour: np.ndarray, depth: np.ndarray, cam_to_world: np.ndarray, fx: float, fy: float,
                   cx: float, cy: float, f: int, prm: FrustumParams, pixels: np.ndarray | None = None) -> FrustumSets:
    """S^f(p) by the definition above. colour [N, H, W, 3], depth [N, H, W] float64."""
    n_frames, h, w = depth.shape
    k = _poses.intrinsics(fx, fy, cx, cy)
    half = prm.l / 2.0
    reach = int(np.ceil(half)) + 1
    if pixels is None:
        pixels = np.arange(h * w, dtype=np.int64)
    pixels = np.asarray(pixels, dtype=np.int64)
    slot = -np.ones(h * w, dtype=np.int64)
    slot[pixels] = np.arange(pixels.size)
    dp = depth[f].reshape(-1)
    parts = []     # (slot, id, rho, colour, marginal) per window frame and offset
    near = []      # (slot, id) of non-members within a band
    near_miss = np.zeros(pixels.size, dtype=bool)
    j_lo, j_hi = max(0, f - prm.window), min(n_frames - 1, f + prm.window)
    for j in range(j_lo, j_hi + 1):
        px, py, z = carried_into_output(depth[j], cam_to_world[j], cam_to_world[f], k)
        with np.errstate(invalid="ignore"):
            ok = np.isfinite(depth[j]) & (depth[j] > 0) & np.isfinite(px) & np.isfinite(py)
            in_z = (z >= prm.near) & (z <= prm.far)
            z_marg = (np.abs(z - prm.near) <= Z_BAND * prm.near) | (np.abs(z - prm.far) <= Z_BAND * prm.far)
        cand = np.flatnonzero((ok & (in_z | z_marg)).ravel())     # source pixels q worth testing
        ax, ay = px.ravel()[cand], py.ravel()[cand]
        zq, inzq, zmq = z.ravel()[cand], in_z.ravel()[cand], z_marg.ravel()[cand]
        bx, by = np.floor(ax).astype(np.int64), np.floor(ay).astype(np.int64)
        # every output pixel within `reach` of the carried point, one offset at a time
        for oy_off in range(-reach, reach + 1):
            for ox_off in range(-reach, reach + 1):
                ox, oy = bx + ox_off, by + oy_off
                inside = (ox >= 0) & (ox < w) & (oy >= 0) & (oy < h)
                at = np.where(inside, oy * w + ox, 0)
                sl = np.where(inside, slot[at], -1)
                use = sl >= 0
                if not use.any():
                    continue
                dist = np.abs(ox - ax) + np.abs(oy - ay)
                marg = zmq | (np.abs(dist - half) <= L1_BAND)
                member = use & (dist < half) & inzq
                nm = use & ~member & marg
                near_miss[sl[nm]] = True
                if nm.any():
                    near.append((sl[nm], ((j - f + prm.window) << ID_SHIFT) | cand[nm]))
                if not member.any():
                    continue
                q = cand[member]
                d_ref = dp[at[member]]
                with np.errstate(invalid="ignore", divide="ignore"):
                    rho = np.where(np.isfinite(d_ref) & (d_ref > 0), (zq[member] - d_ref) / d_ref, np.nan)
                ident = ((j - f + prm.window) << ID_SHIFT) | q
                parts.append((sl[member], ident, rho, colour[j].reshape(-1, 3)[q], marg[member]))
    if parts:
        slots = np.concatenate([p_[0] for p_ in parts])
        idents = np.concatenate([p_[1] for p_ in parts]).astype(np.int64)
        rhos = np.concatenate([p_[2] for p_ in parts])
        cols = np.concatenate([p_[3] for p_ in parts])
        margs = np.concatenate([p_[4] for p_ in parts])
    else:
        slots = idents = np.zeros(0, dtype=np.int64)
        rhos, cols, margs = np.zeros(0), np.zeros((0, 3)), np.zeros(0, dtype=bool)
    order = np.lexsort((idents, slots))      # by output pixel, then ascending id
    counts = np.bincount(slots, minlength=pixels.size)
    offsets = np.zeros(pixels.size + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    if near:
        n_sl = np.concatenate([a for a, _ in near])
        n_id = np.concatenate([b for _, b in near]).astype(np.int64)
    else:
        n_sl = n_id = np.zeros(0, dtype=np.int64)
    n_order = np.lexsort((n_id, n_sl))
    near_offsets = np.zeros(pixels.size + 1, dtype=np.int64)
    near_offsets[1:] = np.cumsum(np.bincount(n_sl, minlength=pixels.size))
    return FrustumSets(frame=f, pixels=pixels, offsets=offsets, ids=idents[order].astype(np.uint32),
                       rho=rhos[order], colour=cols[order].reshape(-1, 3), marginal=margs[order],
                       near_miss=near_miss, near_offsets=near_offsets, near_ids=n_id[n_order].astype(np.uint32))


def _convex_hull(pts: np.ndarray) -> np.ndarray:
    """Counter-clockwise hull (Andrew's monotone chain) of 2D points [m, 2]."""
    p = sorted(set(map(tuple, pts)))
    if len(p) <= 2:
        return np.array(p)

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for pt in p:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], pt) <= 0:
            lower.pop()
        lower.append(pt)
    for pt in reversed(p):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], pt) <= 0:
            upper.pop()
        upper.append(pt)
    return np.array(lower[:-1] + upper[:-1])


def gather_frustum_hull(depth: np.ndarray, cam_to_world: np.ndarray, fx: float, fy: float, cx: float, cy: float,
                        f: int, prm: FrustumParams, p: int) -> list[int]:
    """The paper's algorithm for one output pixel p (flat index): for each window
    frame J, project the 8 corners of V (Eq. 1) into J, take the pixels inside
    (or on) their convex hull, and keep those passing Eq. 2 and the depth range.
    Returns the member ids in ascending order. Requires V in front of every J
    (raises otherwise)."""
    n_frames, h, w = depth.shape
    k = _poses.intrinsics(fx, fy, cx, cy)
    kinv = np.linalg.inv(k)
    half = prm.l / 2.0
    px, py = p % w, p // w
    corners = []
    for sx in (-half, half):
        for sy in (-half, half):
            for d in (prm.near, prm.far):
                corners.append(np.append(d * (kinv @ np.array([px + sx, py + sy, 1.0])), 1.0))
    corners_w = np.array([cam_to_world[f] @ c for c in corners])               # [8, 4]
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    out = []
    for j in range(max(0, f - prm.window), min(n_frames - 1, f + prm.window) + 1):
        cj = np.linalg.inv(cam_to_world[j]) @ corners_w.T                      # [4, 8]
        if np.any(cj[2] <= 0):
            raise ValueError("frustum reaches behind camera J")
        uv = np.stack([k[0, 0] * cj[0] / cj[2] + k[0, 2], k[1, 1] * cj[1] / cj[2] + k[1, 2]], axis=1)
        hull = _convex_hull(uv)
        inside = np.ones((h, w), dtype=bool)
        m = len(hull)
        for a in range(m):                                 # left of (or on) every edge
            e0, e1 = hull[a], hull[(a + 1) % m]
            side = (e1[0] - e0[0]) * (yy - e0[1]) - (e1[1] - e0[1]) * (xx - e0[0])
            inside &= side >= -1e-9 * max(1.0, float(np.abs(uv).max()))
        qx_, qy_, z = carried_into_output(depth[j], cam_to_world[j], cam_to_world[f], k)
        with np.errstate(invalid="ignore"):
            ok = (np.isfinite(depth[j]) & (depth[j] > 0) & inside & (z >= prm.near) & (z <= prm.far)
                  & (np.abs(qx_ - px) + np.abs(qy_ - py) < half))
        for q in np.flatnonzero(ok.ravel()):
            out.append(((j - f + prm.window) << ID_SHIFT) | int(q))
    return sorted(out)
