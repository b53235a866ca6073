"""Sample-set filtering (test infrastructure only).

Sec. 5 Eq. 3: O(p) = (1 / W) sum_{s in S(p)} w(s) s_rgb with W = sum w(s).
Sec. 5 Eq. 4: the denoising weight is a Gaussian around the reference
sample s_ref (the sample that the output pixel itself contributes: frame f,
pixel p) with a diagonal covariance. Here the terms are
  w(s) = exp(-rho_s^2 / (2 sd^2)) * exp(-|c_s - c_ref|^2 / (2 sc^2)) * exp(-(J_s - f)^2 / (2 st^2))
where rho_s is the sample's relative depth residual (the depth-guided gather's
stand-in for the scene-space distance to s_ref), c_ref = I^f(p), and a sigma
of +inf disables its term (weight factor 1). sd alone is the depth-Gaussian
weighted mean; sd = sc = st = inf is the plain mean of Sec. 5 (w = 1).
An empty set returns the input colour I^f(p) (reading: the paper is silent).
"""
from __future__ import annotations

import math

import numpy as np

from .gather import ID_SHIFT, OracleSets


def _factor(dist2: np.ndarray, sigma: float) -> np.ndarray:
    if math.isinf(sigma):
        return np.ones_like(dist2)
    return np.exp(-dist2 / (2.0 * sigma * sigma))


def weighted_mean(offsets: np.ndarray, colour: np.ndarray, rho: np.ndarray, dj: np.ndarray,
                  c_ref: np.ndarray, sigma_d: float, sigma_c: float = math.inf,
                  sigma_t: float = math.inf) -> np.ndarray:
    """Eq. 3 with the weight above over CSR sets; returns [n, 3] float64."""
    n = offsets.size - 1
    counts = np.diff(offsets)
    seg = np.repeat(np.arange(n), counts)
    dc2 = np.sum((colour - c_ref[seg]) ** 2, axis=1)
    w = _factor(rho * rho, sigma_d) * _factor(dc2, sigma_c) * _factor(dj.astype(np.float64) ** 2, sigma_t)
    wsum = np.bincount(seg, weights=w, minlength=n)
    out = np.empty((n, 3))
    for ch in range(3):
        out[:, ch] = np.bincount(seg, weights=w * colour[:, ch], minlength=n)
    empty = counts == 0
    with np.errstate(invalid="ignore", divide="ignore"):
        out = out / wsum[:, None]
    out[empty] = c_ref[empty]
    return out


def filter_sets(sets: OracleSets, colour_f: np.ndarray, window: int, sigma_d: float,
                sigma_c: float = math.inf, sigma_t: float = math.inf) -> np.ndarray:
    """Filter the oracle's own sets; colour_f is the frame-f colour plane [H, W, 3]."""
    c_ref = colour_f.reshape(-1, 3)[sets.pixels]
    dj = (sets.ids.astype(np.int64) >> ID_SHIFT) - window
    return weighted_mean(sets.offsets, sets.colour, sets.rho, dj, c_ref, sigma_d, sigma_c, sigma_t)


# ---------------------------------------------------------------------------
# The paper's other filters over the same sets (Sec. 5).

def frame_weighted_mean(sets: OracleSets, colour_f: np.ndarray, window: int, frame_w: np.ndarray,
                        sigma_d: float, sigma_c: float = math.inf, sigma_t: float = math.inf) -> np.ndarray:
    """Eq. 3 with the weight of Eq. 4 multiplied by a per-source-frame factor
    frame_w[J] (J = the frame the sample came from, absolute index):
      deblurring (Sec. 5, Eq. 5): frame_w[J] = B(J), the frame's summed gradient magnitude;
      computational shutter (Sec. 5, Eq. 10): frame_w[J] = xi(J) with every sigma +inf.
    Reading: a set whose weights sum to zero (empty, or every sample on a frame of
    factor 0) returns the input colour I^f(p). Returns [n, 3] float64."""
    n = sets.offsets.size - 1
    counts = np.diff(sets.offsets)
    seg = np.repeat(np.arange(n), counts)
    c_ref = colour_f.reshape(-1, 3)[sets.pixels]
    dj = (sets.ids.astype(np.int64) >> ID_SHIFT) - window
    src_frame = sets.frame + dj
    dc2 = np.sum((sets.colour - c_ref[seg]) ** 2, axis=1)
    w = (_factor(sets.rho * sets.rho, sigma_d) * _factor(dc2, sigma_c) * _factor(dj.astype(np.float64) ** 2, sigma_t)
         * np.asarray(frame_w, dtype=np.float64)[src_frame])
    wsum = np.bincount(seg, weights=w, minlength=n)
    out = np.empty((n, 3))
    for ch in range(3):
        out[:, ch] = np.bincount(seg, weights=w * sets.colour[:, ch], minlength=n)
    none = wsum == 0.0
    with np.errstate(invalid="ignore", divide="ignore"):
        out = out / wsum[:, None]
    out[none] = c_ref[none]
    return out


def scene_space_weighted_mean(sets: OracleSets, colour_f: np.ndarray, depth: np.ndarray, cam_to_world: np.ndarray,
                              fx: float, fy: float, cx: float, cy: float, window: int, sigma_d: float,
                              sigma_c: float, sigma_xyz: float, sigma_t: float,
                              frame_w: np.ndarray | None = None) -> np.ndarray:
    """Eq. 3 with the full weight of Eq. 4 (Sec. 5, denoising): a Gaussian around the
    reference sample over colour, scene-space position and frame time,
      w(s) = exp(-|c_s - c_ref|^2 / 2 sc^2) exp(-|X_s - X_ref|^2 / 2 sxyz^2) exp(-(J_s - f)^2 / 2 st^2)
    times the depth-residual term exp(-rho_s^2 / 2 sd^2) of the depth-guided gather
    and, when given, a per-source-frame factor frame_w[J] (deblurring, Eq. 5, reuses
    this weight times B(J)). X_s is the sample's scene point, X = C^J [D^J(q) K^-1
    (q_x, q_y, 1), 1] from its source pixel's stored depth, and X_ref that of the
    output pixel p itself (the reference sample s_ref of frame f). A sigma of +inf
    disables its term. sxyz is in world units (the paper states it in units of a
    scene scaled so that 90 % of its points lie in a 10^3 cube; the caller converts).
    Readings: an output pixel without a valid depth has no reference point, so with
    a finite sxyz it returns I^f(p), as does a set whose weights sum to zero.
    depth [N, H, W] float64 (the stored depths), cam_to_world [N, 4, 4]. Returns [n, 3]."""
    n_frames, h, w_img = depth.shape
    n = sets.offsets.size - 1
    counts = np.diff(sets.offsets)
    seg = np.repeat(np.arange(n), counts)
    c_ref = colour_f.reshape(-1, 3)[sets.pixels]
    dj = (sets.ids.astype(np.int64) >> ID_SHIFT) - window
    src = sets.frame + dj
    q = sets.ids.astype(np.int64) & ((1 << ID_SHIFT) - 1)
    dc2 = np.sum((sets.colour - c_ref[seg]) ** 2, axis=1)
    w = _factor(sets.rho * sets.rho, sigma_d) * _factor(dc2, sigma_c) * _factor(dj.astype(np.float64) ** 2, sigma_t)
    if frame_w is not None:
        w = w * np.asarray(frame_w, dtype=np.float64)[src]
    no_ref = np.zeros(n, dtype=bool)
    if not math.isinf(sigma_xyz):
        def world(frames, pix):
            x = (pix % w_img).astype(np.float64)
            y = (pix // w_img).astype(np.float64)
            d = depth[frames, pix // w_img, pix % w_img].astype(np.float64)
            xc = np.stack([d * (x - cx) / fx, d * (y - cy) / fy, d])
            rot = cam_to_world[frames, :3, :3]
            return np.einsum("nij,jn->ni", rot, xc) + cam_to_world[frames, :3, 3], d
        x_ref, d_ref = world(np.full(n, sets.frame), sets.pixels.astype(np.int64))
        no_ref = ~(np.isfinite(d_ref) & (d_ref > 0.0))
        x_s, _ = world(src, q)
        dxyz2 = np.sum((x_s - x_ref[seg]) ** 2, axis=1)
        with np.errstate(invalid="ignore"):
            w = w * _factor(dxyz2, sigma_xyz)
        w[no_ref[seg]] = 0.0
    wsum = np.bincount(seg, weights=w, minlength=n)
    out = np.empty((n, 3))
    for ch in range(3):
        out[:, ch] = np.bincount(seg, weights=w * sets.colour[:, ch], minlength=n)
    none = (wsum == 0.0) | no_ref
    with np.errstate(invalid="ignore", divide="ignore"):
        out = out / wsum[:, None]
    out[none] = c_ref[none]
    return out


def frame_sharpness(colour: np.ndarray) -> np.ndarray:
    """B(J) of Eq. 5: the sum over the pixels q of frame J of |grad I^J(q)|.
    Reading (the paper names the gradient operator only): forward differences
    gx = I(x + 1, y) - I(x, y), gy = I(x, y + 1) - I(x, y) of each colour channel,
    |grad I(q)| = sqrt(sum over channels of gx^2 + gy^2), summed over the pixels
    whose right and lower neighbours lie in the image. colour [N, H, W, 3] -> [N]."""
    c = np.asarray(colour, dtype=np.float64)
    gx = c[:, :-1, 1:, :] - c[:, :-1, :-1, :]
    gy = c[:, 1:, :-1, :] - c[:, :-1, :-1, :]
    mag = np.sqrt(np.sum(gx * gx + gy * gy, axis=3))
    return mag.reshape(c.shape[0], -1).sum(axis=1)


def inpaint_mean_shift(sets: OracleSets, colour_f: np.ndarray, window: int, mask: np.ndarray,
                       sigma_rgb: float, steps: int = 2, sigma_ref: float = math.inf) -> np.ndarray:
    """Inpainting (Sec. 5, Eq. 8-9) for the output pixels of frame sets.frame.

    mask [N, H, W] bool: M^J(q), True = the pixel shows content to remove.
    For an output pixel with M^f(p) = 1: s_ref starts as the mean colour of all
    samples of S(p) (Eq. 8); each step replaces it with the weighted mean of the
    samples, weight exp(-|s_ref - c_s|^2 / (2 sigma_rgb^2)) for a sample whose
    source pixel is unmasked and 0 for a masked one (Eq. 9); the output is s_ref
    after `steps` steps (the paper uses two). Readings: only the colour dimensions
    are used (the paper gives sigma_rgb alone); the initial mean takes every sample,
    masked ones included, as Eq. 8 is written; an unmasked output pixel, an empty
    set, or a step whose weights sum to zero returns I^f(p). Returns [n, 3] float64.

    Semi-transparency (same paragraph): with a finite sigma_ref every weight is also
    multiplied by exp(-|c_s - I^f(p)|^2 / (2 sigma_ref^2)), the standard weighting
    around the input pixel, which favours samples coloured like the object being
    made transparent (the paper uses sigma_rgb = 80 for it). Reading: the factor
    multiplies the inpainting weight of every step; the initial mean is unchanged."""
    h, w_img = colour_f.shape[:2]
    c_ref = colour_f.reshape(-1, 3)[sets.pixels]
    dj = (sets.ids.astype(np.int64) >> ID_SHIFT) - window
    q = (sets.ids.astype(np.int64) & ((1 << ID_SHIFT) - 1))
    src_masked = np.asarray(mask, dtype=bool).reshape(mask.shape[0], -1)[sets.frame + dj, q]
    out_masked = np.asarray(mask, dtype=bool)[sets.frame].reshape(-1)[sets.pixels]
    out = c_ref.copy()
    for i in range(sets.pixels.size):
        a, b = sets.offsets[i], sets.offsets[i + 1]
        if not out_masked[i] or b == a:
            continue
        cs = sets.colour[a:b]
        keep = ~src_masked[a:b]
        s_ref = cs.mean(axis=0)
        to_input = _factor(np.sum((cs - c_ref[i]) ** 2, axis=1), sigma_ref)
        ok = True
        for _ in range(steps):
            wgt = np.where(keep, np.exp(-np.sum((cs - s_ref) ** 2, axis=1) / (2.0 * sigma_rgb * sigma_rgb)), 0.0)
            wgt = wgt * to_input
            tot = wgt.sum()
            if tot == 0.0:
                ok = False
                break
            s_ref = (wgt[:, None] * cs).sum(axis=0) / tot
        if ok:
            out[i] = s_ref
    return out


def scene_points(depth: np.ndarray, cam_to_world: np.ndarray, fx: float, fy: float, cx: float,
                 cy: float) -> np.ndarray:
    """World position of every pixel q = (x, y) of every frame J (Sec. 3: a pixel
    with its depth and camera matrix is a scene point): X_cam = d ((x - cx) / fx,
    (y - cy) / fy, 1), X = R^J X_cam + t^J with C^J = [R^J | t^J], each sum taken
    left to right. depth [N, H, W] -> [N, H, W, 3] float64."""
    n, h, w = depth.shape
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    out = np.empty((n, h, w, 3))
    for j in range(n):
        d = np.asarray(depth[j], dtype=np.float64)
        xc, yc, zc = d * ((xx - cx) / fx), d * ((yy - cy) / fy), d
        c = np.asarray(cam_to_world[j], dtype=np.float64)
        for k in range(3):
            out[j, :, :, k] = ((c[k, 0] * xc + c[k, 1] * yc) + c[k, 2] * zc) + c[k, 3]
    return out


def scene_box_mask(depth: np.ndarray, cam_to_world: np.ndarray, fx: float, fy: float, cx: float, cy: float,
                   lo, hi) -> np.ndarray:
    """Inpainting masks from a scene-space region (Sec. 5, inpainting: the samples
    inside the region, projected back into the images, form M). Reading: the region
    is an axis-aligned box [lo, hi] in world coordinates, bounds included; a pixel
    without a valid depth (not finite, or <= 0) is not a scene point and stays
    unmasked. Returns [N, H, W] bool."""
    d = np.asarray(depth, dtype=np.float64)
    with np.errstate(invalid="ignore"):   # inf depths give NaN positions; they are masked out below
        pts = scene_points(d, cam_to_world, fx, fy, cx, cy)
        ok = np.isfinite(d) & (d > 0.0)
        inside = np.ones(d.shape, dtype=bool)
        for k in range(3):
            inside &= (pts[..., k] >= lo[k]) & (pts[..., k] <= hi[k])
    return ok & inside
