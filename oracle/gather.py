"""Sample sets S^f(p) by the depth-guided frustum test (test infrastructure only).

Follows Sec. 4 of the paper. The paper's pixel frustum (Eq. 1) spans the
near..far depth range and its projection V_J into frame J is tested pixel by
pixel with the back-projection check of Eq. 2. The depth-guided variant used
here bounds the frustum by the output pixel's own depth d_p, so its projection
into J collapses to the l x l pixel block (l = 2r + 1, l = 3 in Sec. 4) around
the projected point, and the back-projection check becomes a depth-consistency
check in J: source pixel q is kept when its depth agrees with the predicted
depth of the 3D point to a relative tolerance tau.

Definition, for output frame f and pixel p = (x, y) (x column, y row):
  1. d_p = D^f(p). If d_p is not finite or d_p <= z_near, S = {}.
  2. X = d_p K^{-1} [x, y, 1]^T   (camera-f coordinates).
  3. For each J in [max(0, f - w), min(N - 1, f + w)], ascending:
       (R, t) = T_{J<-f} = inv(C^J) C^f   (exact identity for J = f);
       Y = R X + t, z = Y_3; skip J if z <= z_near;
       u = fx Y_1 / z + cx, v = fy Y_2 / z + cy; u^ = floor(u + 1/2), v^ = floor(v + 1/2);
       for dy = -r..r, then dx = -r..r: q = (u^ + dx, v^ + dy), skipped when
       outside the image or when d_q = D^J(q) is not finite or d_q <= 0;
       rho = (d_q - z) / z; q is a member iff |rho| <= tau.
  4. Member id = ((J - f + w) << 22) | (q_y W + q_x); members are listed in
     ascending id (J ascending, then the block in row-major order).

Reading notes (the paper is silent on these): the window is truncated, not
shifted, at clip ends and includes J = f; out-of-image block pixels are
dropped; tau scales the predicted depth z.

Parity bands: results computed in float32 may legitimately differ from this
float64 definition where the decision sits on a threshold. Each member or
candidate within a band is flagged so a comparison can exempt exactly those:
  * depth band:   | |rho| - tau | <= RHO_BAND;
  * rounding band: u or v within EPS_PX of a half-integer (the whole block of
    both roundings is exempt);
  * near band:    |z - z_near| <= NEAR_BAND * z_near.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import poses as _poses

RHO_BAND = 1e-5
# float32 projections are off by up to 9e-4 px in u, v (the folded float32 map,
# the approximate reciprocal and the rounded u + 1/2) and 2e-7 in relative z at
# 1920x1080 with the full-scale workload's poses over +-50 frames
# (tests/test_float32_bands.py): the bands are at least eight times that
EPS_PX = 2.0 ** -7
NEAR_BAND = 1e-5
ID_SHIFT = 22


@dataclass
class GatherParams:
    window: int
    radius: int = 1
    tol: float = 0.01
    z_near: float = 0.01


@dataclass
class OracleSets:
    """Sets for a list of output pixels of frame `frame`.

    members (CSR over the pixel list): ids, rho, colour, marginal flag.
    maybe   (CSR over the pixel list): ids (and rho) of non-members that a
            float32 evaluation may legitimately include.
    """
    frame: int
    pixels: np.ndarray         # [n] flat indices y * W + x
    offsets: np.ndarray        # [n + 1] int64
    ids: np.ndarray            # [S] uint32
    rho: np.ndarray            # [S] float64
    colour: np.ndarray         # [S, 3] float64
    marginal: np.ndarray       # [S] bool
    maybe_offsets: np.ndarray  # [n + 1] int64
    maybe_ids: np.ndarray      # [M] uint32
    maybe_rho: np.ndarray      # [M] float64

    def members_of(self, i: int) -> np.ndarray:
        return self.ids[self.offsets[i]:self.offsets[i + 1]]


def make_id(dj: np.ndarray, window: int, q_flat: np.ndarray) -> np.ndarray:
    return ((dj + window).astype(np.uint64) << np.uint64(ID_SHIFT)) | q_flat.astype(np.uint64)


def project(depth_p: np.ndarray, x: np.ndarray, y: np.ndarray, t_rel: np.ndarray, k: np.ndarray):
    """Step 2-3: (u, v, z) of the pixels (x, y) with depth depth_p seen from frame J."""
    kinv = np.linalg.inv(k)
    pix = np.stack([x, y, np.ones_like(x)], axis=0).astype(np.float64)      # [3, n]
    xcam = depth_p[None, :] * (kinv @ pix)                                   # X, [3, n]
    ycam = t_rel[:3, :3] @ xcam + t_rel[:3, 3:4]                             # Y, [3, n]
    z = ycam[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = k[0, 0] * ycam[0] / z + k[0, 2]
        v = k[1, 1] * ycam[1] / z + k[1, 2]
    return u, v, z


def gather_frame(colour: np.ndarray, depth: np.ndarray, cam_to_world: np.ndarray,
                 fx: float, fy: float, cx: float, cy: float, f: int, prm: GatherParams,
                 pixels: np.ndarray | None = None) -> OracleSets:
    """S^f(p) for `pixels` (default: every pixel of frame f).

    colour [N, H, W, 3] and depth [N, H, W] are float64 (already rounded the way
    the comparison needs, e.g. mode Q); cam_to_world [N, 4, 4].
    """
    n_frames, h, w_img = depth.shape
    k = _poses.intrinsics(fx, fy, cx, cy)
    r, tau, zn, win = prm.radius, prm.tol, prm.z_near, prm.window
    if pixels is None:
        pixels = np.arange(h * w_img, dtype=np.int64)
    pixels = np.asarray(pixels, dtype=np.int64)
    n = pixels.size
    x = (pixels % w_img).astype(np.float64)
    y = (pixels // w_img).astype(np.float64)
    dp = depth[f].reshape(-1)[pixels]
    with np.errstate(invalid="ignore"):
        valid_p = np.isfinite(dp) & (dp > zn)
    pos_all = np.arange(n, dtype=np.int64)

    parts = []  # (pos, id, rho, colour, member, marginal, alt)
    j_lo, j_hi = max(0, f - win), min(n_frames - 1, f + win)
    for j in range(j_lo, j_hi + 1):
        t_rel = _poses.relative(cam_to_world[f], cam_to_world[j], same_frame=(j == f))
        u, v, z = project(np.where(valid_p, dp, 1.0), x, y, t_rel, k)
        near_marg = valid_p & (np.abs(z - zn) <= NEAR_BAND * zn)
        z_ok = valid_p & (z > zn)
        with np.errstate(invalid="ignore"):
            uf, vf = np.floor(u), np.floor(v)
            u_marg = np.abs(u - (uf + 0.5)) <= EPS_PX
            v_marg = np.abs(v - (vf + 0.5)) <= EPS_PX
            uh, vh = np.floor(u + 0.5), np.floor(v + 0.5)
        pair_marg = near_marg | u_marg | v_marg
        dplane = depth[j].reshape(-1)
        cplane = colour[j].reshape(-1, 3)
        # rounding alternatives: (u option, v option, is_alternative)
        options = [(uh, vh, z_ok, False)]
        enum_any = z_ok | near_marg
        ua = np.where(uh == uf, uf + 1.0, uf)
        va = np.where(vh == vf, vf + 1.0, vf)
        options.append((ua, vh, enum_any & u_marg, True))
        options.append((uh, va, enum_any & v_marg, True))
        options.append((ua, va, enum_any & u_marg & v_marg, True))
        options.append((uh, vh, near_marg & ~z_ok, True))  # float32 may see z > z_near
        for (uo, vo, sel, is_alt) in options:
            if not sel.any():
                continue
            idx = pos_all[sel]
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    qx = uo[sel] + dx
                    qy = vo[sel] + dy
                    inb = (qx >= 0) & (qx < w_img) & (qy >= 0) & (qy < h)
                    if not inb.any():
                        continue
                    ii = idx[inb]
                    qf = (qy[inb] * w_img + qx[inb]).astype(np.int64)
                    dq = dplane[qf]
                    zz = z[ii]
                    with np.errstate(invalid="ignore", divide="ignore"):
                        rho = (dq - zz) / zz
                        dq_ok = np.isfinite(dq) & (dq > 0.0)
                        arho = np.abs(rho)
                        band = np.abs(arho - tau) <= RHO_BAND
                        member = dq_ok & (arho <= tau) & (not is_alt)
                        loose = dq_ok & (arho <= tau + RHO_BAND)
                    keep = member | loose
                    if not keep.any():
                        continue
                    ids = make_id(np.full(keep.sum(), j - f), win, qf[keep])
                    marg = band[keep] | pair_marg[ii[keep]] | np.bool_(is_alt)
                    parts.append((ii[keep], ids, rho[keep], cplane[qf[keep]], member[keep], marg, is_alt))

    if parts:
        pos = np.concatenate([p[0] for p in parts])
        ids = np.concatenate([p[1] for p in parts])
        rho = np.concatenate([p[2] for p in parts])
        col = np.concatenate([p[3] for p in parts])
        mem = np.concatenate([p[4] for p in parts])
        mar = np.concatenate([p[5] for p in parts])
        alt = np.concatenate([np.full(p[0].size, p[6]) for p in parts])
    else:
        pos = np.zeros(0, np.int64)
        ids = np.zeros(0, np.uint64)
        rho = np.zeros(0)
        col = np.zeros((0, 3))
        mem = mar = alt = np.zeros(0, bool)
    # canonical order: pixel, then id; a primary evaluation wins over an alternative one
    order = np.lexsort((alt, ids, pos))
    pos, ids, rho, col, mem, mar, alt = pos[order], ids[order], rho[order], col[order], mem[order], mar[order], alt[order]
    if pos.size:
        first = np.ones(pos.size, bool)
        first[1:] = (pos[1:] != pos[:-1]) | (ids[1:] != ids[:-1])
        pos, ids, rho, col, mem, mar = pos[first], ids[first], rho[first], col[first], mem[first], mar[first]

    m_sel = mem
    y_sel = ~mem
    offsets = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(pos[m_sel], minlength=n), out=offsets[1:])
    moff = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(pos[y_sel], minlength=n), out=moff[1:])
    return OracleSets(
        frame=f, pixels=pixels, offsets=offsets,
        ids=ids[m_sel].astype(np.uint32), rho=rho[m_sel], colour=col[m_sel], marginal=mar[m_sel],
        maybe_offsets=moff, maybe_ids=ids[y_sel].astype(np.uint32), maybe_rho=rho[y_sel],
    )
