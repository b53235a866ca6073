"""Comparison helpers: HIP sample sets / filtered colours vs the float64 oracle.

The contract (membership bit-exact outside the oracle's bands, colours within
1e-3 on the 0-1 scale) is spelled out in each function.
"""
from __future__ import annotations

import numpy as np

from oracle import filters as ofilters
from oracle import gather as ogather

ID_MASK = (1 << 22) - 1
COLOUR_TOL = 1e-3          # filtered colour, 0-1 scale
FILTER_ARITH_TOL = 2e-5    # same records, float32 vs float64 arithmetic


def f16_to_f64(a_u16: np.ndarray) -> np.ndarray:
    return a_u16.view(np.float16).astype(np.float64)


def gpu_sets_to_host(sets, frame_index: int, n_pix_frame: int):
    """Slice output frame `frame_index` (0-based within the call) out of GPU sets."""
    off = sets.offsets.cpu().numpy()
    lo, hi = frame_index * n_pix_frame, (frame_index + 1) * n_pix_frame
    o = off[lo:hi + 1]
    ids = sets.ids[o[0]:o[-1]].cpu().numpy().view(np.uint32)
    crho = sets.crho[o[0]:o[-1]].cpu().numpy().view(np.uint16)
    return o - o[0], ids, crho


def compare_membership(orc: ogather.OracleSets, g_off, g_ids, g_crho, rgbd_u16: np.ndarray, f: int,
                       window: int, pixels=None):
    """Check certain members <= GPU set <= members + maybe, canonical order,
    record colours bit-exact, rho within binary16 rounding.

    rgbd_u16: [N, H, W, 4] uint16 staged planes (as stored on the GPU).
    pixels: the oracle's pixel list when it is a subset (GPU sets are sliced to it).
    Returns a dict of statistics.
    """
    n_frames, h, w = rgbd_u16.shape[:3]
    if pixels is not None:
        counts = np.diff(g_off)[pixels]
        starts = g_off[pixels]
        sel = np.concatenate([np.arange(s, s + c) for s, c in zip(starts, counts)]) if counts.sum() else np.zeros(0, np.int64)
        g_ids_s, g_crho_s = g_ids[sel], g_crho[sel]
        g_off_s = np.zeros(len(pixels) + 1, np.int64)
        np.cumsum(counts, out=g_off_s[1:])
    else:
        g_off_s, g_ids_s, g_crho_s = g_off, g_ids, g_crho
    n = g_off_s.size - 1
    seg_g = np.repeat(np.arange(n, dtype=np.uint64), np.diff(g_off_s))
    key_g = (seg_g << np.uint64(32)) | g_ids_s.astype(np.uint64)
    # canonical order: strictly increasing (pixel, id)
    assert np.all(np.diff(key_g.astype(np.int64)) > 0) if key_g.size > 1 else True, "records not in canonical order"

    seg_o = np.repeat(np.arange(n, dtype=np.uint64), np.diff(orc.offsets))
    key_o = (seg_o << np.uint64(32)) | orc.ids.astype(np.uint64)
    seg_m = np.repeat(np.arange(n, dtype=np.uint64), np.diff(orc.maybe_offsets))
    key_m = (seg_m << np.uint64(32)) | orc.maybe_ids.astype(np.uint64)
    certain = key_o[~orc.marginal]
    missing = ~np.isin(certain, key_g)
    assert not missing.any(), f"{missing.sum()} certain members missing from the GPU sets"
    allowed = np.concatenate([key_o, key_m])
    extra = ~np.isin(key_g, allowed)
    assert not extra.any(), f"{extra.sum()} GPU records are not members"

    # record colours: exact copies of the stored source pixel
    dj = (g_ids_s >> 22).astype(np.int64) - window
    q = (g_ids_s & ID_MASK).astype(np.int64)
    j = f + dj
    assert np.all((j >= 0) & (j < n_frames)) and np.all(q < h * w)
    src = rgbd_u16.reshape(n_frames, h * w, 4)[j, q]
    assert np.array_equal(src[:, :3], g_crho_s[:, :3]), "record colour differs from the source pixel"

    # rho: binary16 rounding of the float32 residual
    rho_g = f16_to_f64(g_crho_s[:, 3].copy())
    all_rho = np.concatenate([orc.rho, orc.maybe_rho])
    order = np.argsort(allowed)
    pos = np.searchsorted(allowed[order], key_g)
    rho_o = all_rho[order][pos]
    err = np.abs(rho_g - rho_o)
    lim = np.abs(rho_o) * 2.0 ** -11 + 2.0 ** -25 + 1e-6
    assert np.all(err <= lim), f"rho error {err.max():.3g}"
    return {
        "records": int(key_g.size),
        "oracle_members": int(key_o.size),
        "marginal": int(orc.marginal.sum()),
        "maybe": int(key_m.size),
        "gpu_marginal_diff": int((~np.isin(key_o, key_g)).sum() + (~np.isin(key_g, key_o)).sum()),
        "max_rho_err": float(err.max()) if err.size else 0.0,
    }


def filter_from_records(g_off, g_ids, g_crho, c_ref, window, sigma_d, sigma_c=np.inf, sigma_t=np.inf):
    """The oracle's float64 Eq. 3 applied to the GPU's own records (as stored)."""
    col = f16_to_f64(g_crho[:, :3].copy())
    rho = f16_to_f64(g_crho[:, 3].copy())
    dj = (g_ids >> 22).astype(np.int64) - window
    return ofilters.weighted_mean(g_off, col, rho, dj, c_ref, sigma_d, sigma_c, sigma_t)


def pixels_with_band_cases(orc: ogather.OracleSets) -> np.ndarray:
    """Boolean per oracle pixel: the set holds a marginal member or a maybe candidate."""
    n = orc.offsets.size - 1
    seg = np.repeat(np.arange(n), np.diff(orc.offsets))
    flag = np.zeros(n, bool)
    flag[seg[orc.marginal]] = True
    flag |= np.diff(orc.maybe_offsets) > 0
    return flag


def compare_frustum(orc, g_off, g_ids, g_crho, dp):
    """Frustum sets, candidate by candidate: for every listed output pixel, the
    oracle's members outside its bands are in the GPU's set, every GPU id is an
    oracle member or one of its near-miss non-members, ids ascend, and each shared
    member carries the source pixel's colour exactly and rho within binary16 rounding
    (NaN when the pixel has no valid depth). dp: stored depth of each listed pixel.
    Returns counts for the report."""
    members_checked = extra = 0
    for k, i in enumerate(orc.pixels):
        a, b = g_off[i], g_off[i + 1]
        got = g_ids[a:b]
        assert np.all(np.diff(got.astype(np.int64)) > 0), i
        c, d = orc.offsets[k], orc.offsets[k + 1]
        ids = orc.ids[c:d]
        certain = ids[~orc.marginal[c:d]]
        near = orc.near_ids[orc.near_offsets[k]:orc.near_offsets[k + 1]]
        assert np.all(np.isin(certain, got)), i
        assert np.all(np.isin(got, np.concatenate([ids, near]))), i
        shared, gi, oi = np.intersect1d(got, ids, assume_unique=True, return_indices=True)
        assert np.array_equal(f16_to_f64(g_crho[a + gi, :3].copy()), orc.colour[c + oi]), i
        got_rho = f16_to_f64(g_crho[a + gi, 3].copy())
        want = orc.rho[c + oi]
        if np.isfinite(dp[k]) and dp[k] > 0:
            assert np.all(np.abs(got_rho - want) <= 2.0 ** -11 * np.abs(want) + 1e-5), i
        else:
            assert np.isnan(got_rho).all(), i
        members_checked += shared.size
        extra += got.size - shared.size
    return {"pixels": int(orc.pixels.size), "members_checked": members_checked, "near_miss_members_on_gpu": extra,
            "marginal": int(orc.marginal.sum())}
