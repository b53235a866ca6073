"""Data-term-only multi-view depth (Sec. 3, preprocessing) -- test infrastructure only.

For each pixel p of frame f the paper searches along the epipolar lines of the
frames in a temporal window and keeps the depth with the lowest average cost, the
cost being the sum of squared RGB differences over 3x3 patches; there is no
smoothness term. Readings (the paper names only the data term and the patch):
  - the search runs over a given list of depth hypotheses d_k (each one a point on
    every epipolar line at once);
  - for hypothesis d, p's scene point X = C^f [d K^-1 (p_x, p_y, 1), 1] is projected
    into frame J and rounded to the nearest pixel q_J; the patch cost is
    sum over the 3x3 offsets o of |I^f(p + o) - I^J(q_J + o)|^2 (RGB);
  - a frame J counts for d when X lies in front of it (depth > 0) and both patches
    lie inside their images; cost(d) is the mean over the counted frames, and a
    hypothesis no frame counts for is not a candidate;
  - D(p) = the hypothesis of least cost, the lowest index on ties; NaN when p has no
    candidate (its own patch leaves the image, or no frame sees it); a hypothesis
    that is not finite and positive is not a candidate.
For comparisons with a float32 evaluation, `estimate_depth` also flags pixels
whose decision float32 may take differently: a projection within `rnd_band`
pixels of a rounding boundary (a half-integer; the default suits 1080p
coordinates), or a best cost within COST_BAND (relative) of a different cost of
another candidate (equal costs come from equal patches and tie alike in float32).
"""
from __future__ import annotations

import numpy as np

from . import poses as _poses

# float32 projections of the hypotheses are off by up to 4.9e-4 px at 1920x1080
# (full-scale workload's poses, +-2 frames, 1-30 m; tests/test_float32_bands.py):
# the rounding band is six times that
RND_BAND = 3e-3
COST_BAND = 1e-4


def patch_ssd(a: np.ndarray, ay: int, ax: int, b: np.ndarray, by: int, bx: int) -> float:
    """Sum of squared RGB differences of the 3x3 patches centred at (ax, ay) in a and (bx, by) in b."""
    pa = a[ay - 1:ay + 2, ax - 1:ax + 2, :]
    pb = b[by - 1:by + 2, bx - 1:bx + 2, :]
    return float(np.sum((pa - pb) ** 2))


def estimate_depth(colour: np.ndarray, cam_to_world: np.ndarray, fx: float, fy: float, cx: float, cy: float,
                   f: int, window: int, hypotheses: np.ndarray, with_bands: bool = False,
                   rnd_band: float = RND_BAND, pixels: np.ndarray | None = None):
    """D^f and the least average cost per pixel, [H, W] each (float64), and with
    with_bands the band flags [H, W] bool. colour [N, H, W, 3]; the frames J != f in
    [f - window, f + window] are searched. With `pixels` (flat indices y W + x) only
    those pixels are estimated; the others stay NaN / inf / unflagged."""
    n, h, w = colour.shape[:3]
    k = _poses.intrinsics(fx, fy, cx, cy)
    kinv = np.linalg.inv(k)
    others = [j for j in range(max(0, f - window), min(n - 1, f + window) + 1) if j != f]
    to_j = {j: np.linalg.inv(cam_to_world[j]) @ cam_to_world[f] for j in others}
    depth = np.full((h, w), np.nan)
    best = np.full((h, w), np.inf)
    band = np.zeros((h, w), dtype=bool)
    todo = np.arange(h * w) if pixels is None else np.asarray(pixels, dtype=np.int64)
    for y, x in zip(todo // w, todo % w):
        y, x = int(y), int(x)
        if 1 <= x < w - 1 and 1 <= y < h - 1:
            ray = kinv @ np.array([x, y, 1.0])
            all_costs = []
            for d in hypotheses:
                if not (np.isfinite(d) and d > 0):
                    continue
                xf = np.append(d * ray, 1.0)
                costs = []
                for j in others:
                    yj = to_j[j] @ xf
                    if yj[2] <= 0:
                        continue
                    u = k[0, 0] * yj[0] / yj[2] + k[0, 2]
                    v = k[1, 1] * yj[1] / yj[2] + k[1, 2]
                    for c_ in (u, v):
                        if abs(c_ + 0.5 - np.floor(c_ + 0.5)) <= rnd_band or abs(c_ + 0.5 - np.ceil(c_ + 0.5)) <= rnd_band:
                            band[y, x] = True
                    qx, qy = int(np.floor(u + 0.5)), int(np.floor(v + 0.5))
                    if 1 <= qx < w - 1 and 1 <= qy < h - 1:
                        costs.append(patch_ssd(colour[f], y, x, colour[j], qy, qx))
                if costs:
                    c = float(np.mean(costs))
                    all_costs.append(c)
                    if c < best[y, x]:
                        best[y, x] = c
                        depth[y, x] = d
            if len(all_costs) > 1:
                lo = min(all_costs)
                gaps = [c - lo for c in all_costs if c > lo]
                if gaps and min(gaps) <= COST_BAND * max(lo, 1e-30):
                    band[y, x] = True
    if with_bands:
        return depth, best, band
    return depth, best


def cost_intervals(colour: np.ndarray, cam_to_world: np.ndarray, fx: float, fy: float, cx: float, cy: float,
                   f: int, window: int, hypotheses: np.ndarray, pixels: np.ndarray,
                   rnd_band: float = RND_BAND) -> tuple[np.ndarray, np.ndarray]:
    """For comparisons with a float32 evaluation: per listed pixel and hypothesis, the
    range [lo, hi] of mean costs over every rounding that float32 may take. A
    projection within rnd_band of a half-integer may round to either neighbour, so
    the frame's patch cost is the least or largest SSD over those positions; when a
    possible position changes whether the frame counts (its patch leaves the image),
    the hypothesis is left open, [0, inf]. A hypothesis that no frame counts for (in
    every rounding) gets [nan, nan]; the pixel's own patch outside the image gives
    nan throughout. Same definitions as estimate_depth. Returns lo, hi [n, K]."""
    n, h, w = colour.shape[:3]
    k = _poses.intrinsics(fx, fy, cx, cy)
    kinv = np.linalg.inv(k)
    others = [j for j in range(max(0, f - window), min(n - 1, f + window) + 1) if j != f]
    to_j = {j: np.linalg.inv(cam_to_world[j]) @ cam_to_world[f] for j in others}
    pixels = np.asarray(pixels, dtype=np.int64)
    lo = np.full((pixels.size, len(hypotheses)), np.nan)
    hi = np.full((pixels.size, len(hypotheses)), np.nan)

    def roundings(c):
        r = int(np.floor(c + 0.5))
        out = {r}
        if abs(c + 0.5 - np.floor(c + 0.5)) <= rnd_band:
            out.add(r - 1)
        if abs(c + 0.5 - np.ceil(c + 0.5)) <= rnd_band:
            out.add(r + 1)
        return out

    for i, p in enumerate(pixels):
        y, x = int(p // w), int(p % w)
        if not (1 <= x < w - 1 and 1 <= y < h - 1):
            continue
        ray = kinv @ np.array([x, y, 1.0])
        for kk, d in enumerate(hypotheses):
            if not (np.isfinite(d) and d > 0):
                continue
            xf = np.append(d * ray, 1.0)
            lo_sum = hi_sum = 0.0
            counted, open_ = 0, False
            for j in others:
                yj = to_j[j] @ xf
                if yj[2] <= 0:
                    continue
                u = k[0, 0] * yj[0] / yj[2] + k[0, 2]
                v = k[1, 1] * yj[1] / yj[2] + k[1, 2]
                pos = [(qx, qy) for qx in roundings(u) for qy in roundings(v)]
                ins = [1 <= qx < w - 1 and 1 <= qy < h - 1 for qx, qy in pos]
                if any(ins) and not all(ins):
                    open_ = True
                    break
                if not ins[0]:
                    continue
                ssd = [patch_ssd(colour[f], y, x, colour[j], qy, qx) for qx, qy in pos]
                lo_sum += min(ssd)
                hi_sum += max(ssd)
                counted += 1
            if open_:
                lo[i, kk], hi[i, kk] = 0.0, np.inf
            elif counted:
                lo[i, kk], hi[i, kk] = lo_sum / counted, hi_sum / counted
    return lo, hi
