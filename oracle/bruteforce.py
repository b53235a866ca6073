"""All-pairs twin of the gather, in pure Python loops (tiny inputs only).

Test infrastructure only. It restates Sec. 4's test without any of the
shortcuts of `gather`: each output pixel is lifted to a world point with the
4x4 camera matrix C^f (Sec. 3), every source frame's camera matrix is inverted
by Gauss-Jordan elimination written out here, the point is projected into J,
and then EVERY pixel q of J is visited and accepted when it lies in the l x l
block around the rounded projection, inside the image, with a finite positive
depth that agrees with the predicted depth to the relative tolerance. No
relative-pose folding, no neighbourhood enumeration, no vectorisation.
"""
from __future__ import annotations

import math


def _inverse4(m):
    a = [list(map(float, row)) + [1.0 if i == j else 0.0 for j in range(4)] for i, row in enumerate(m)]
    for c in range(4):
        piv = max(range(c, 4), key=lambda r: abs(a[r][c]))
        a[c], a[piv] = a[piv], a[c]
        d = a[c][c]
        a[c] = [e / d for e in a[c]]
        for r in range(4):
            if r != c and a[r][c] != 0.0:
                fct = a[r][c]
                a[r] = [er - fct * ec for er, ec in zip(a[r], a[c])]
    return [row[4:] for row in a]


def _matvec(m, v):
    return [sum(m[i][k] * v[k] for k in range(4)) for i in range(4)]


def gather_all_pairs(depth, cam_to_world, fx, fy, cx, cy, f, window, radius, tol, z_near):
    """Return {pixel_flat: sorted list of (id, rho)} for output frame f.

    depth: nested lists or array [N][H][W] of floats; cam_to_world [N][4][4].
    """
    n_frames = len(depth)
    h = len(depth[0])
    w_img = len(depth[0][0])
    inv = [_inverse4(cam_to_world[j]) for j in range(n_frames)]
    out = {}
    for y in range(h):
        for x in range(w_img):
            dp = float(depth[f][y][x])
            members = []
            if math.isfinite(dp) and dp > z_near:
                xc = [dp * (x - cx) / fx, dp * (y - cy) / fy, dp, 1.0]
                xw = _matvec(cam_to_world[f], xc)
                for j in range(max(0, f - window), min(n_frames - 1, f + window) + 1):
                    yc = _matvec(inv[j], xw)
                    z = yc[2]
                    if not z > z_near:
                        continue
                    u = fx * yc[0] / z + cx
                    v = fy * yc[1] / z + cy
                    uh, vh = math.floor(u + 0.5), math.floor(v + 0.5)
                    for qy in range(h):
                        for qx in range(w_img):
                            if abs(qx - uh) > radius or abs(qy - vh) > radius:
                                continue
                            dq = float(depth[j][qy][qx])
                            if not (math.isfinite(dq) and dq > 0.0):
                                continue
                            rho = (dq - z) / z
                            if abs(rho) <= tol:
                                members.append((((j - f + window) << 22) | (qy * w_img + qx), rho))
            out[y * w_img + x] = sorted(members)
    return out
