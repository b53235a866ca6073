"""GPU parity of the depth-agnostic frustum gather (Sec. 4, Eq. 1-2) through the C
ABI against the float64 oracle's definition; all inputs seeded and synthetic."""
import numpy as np
import pytest
import torch

from oracle import filters as ofilters
from oracle import frustum as ofr
from oracle import staging as ostaging
from scenegen import configs, generate

from tests import parity

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2102_03011_amd as sg
    return sg


def _stage(clip):
    sg = _sg()
    return sg.scene_stage(clip.rgb_u8.to("cuda").contiguous(), clip.depth.to("cuda").contiguous(),
                          clip.cam_to_world.to("cuda").contiguous(), clip.fx, clip.fy, clip.cx, clip.cy)


def _ragged_invalid(clip):
    d = clip.depth.clone()
    m = torch.rand(d.shape, generator=torch.Generator().manual_seed(5))
    d[m < 0.03] = float("nan")
    d[(m >= 0.03) & (m < 0.05)] = 0.0
    d[(m >= 0.05) & (m < 0.06)] = float("inf")
    d[(m >= 0.06) & (m < 0.07)] = 0.005
    clip.depth = d
    return clip


def _case(name):
    if name == "small":
        wl = configs.tiny(seed=4, width=64, height=48, n_frames=5, window=2)
        clip, f = generate(wl.spec), 2
    else:
        wl = configs.tiny(seed=9, width=100, height=37, n_frames=7, window=3, pose_rot_deg=1.0, pose_trans_m=0.03)
        clip, f = _ragged_invalid(generate(wl.spec)), 3
    staged = _stage(clip)
    col = ostaging.colour_q(clip.rgb_u8.cpu().numpy())
    dep = ostaging.depth_q(clip.depth.cpu().numpy())
    orc = ofr.gather_frustum(col, dep, clip.cam_to_world.numpy(), clip.fx, clip.fy, clip.cx, clip.cy, f,
                             ofr.FrustumParams(window=wl.window))
    return wl, clip, staged, col, dep, f, orc


@pytest.fixture(scope="module", params=["small", "ragged"])
def case(request):
    return _case(request.param)


def _unsure(orc):
    seg = np.repeat(np.arange(orc.offsets.size - 1), np.diff(orc.offsets))
    u = orc.near_miss.copy()
    u[seg[orc.marginal]] = True
    return u


def test_frustum_sets_match_oracle(case):
    wl, clip, staged, col, dep, f, orc = case
    sg = _sg()
    h, w = clip.height, clip.width
    sets = sg.scene_gather_frustum(staged, f, sg.FrustumParams(window=wl.window))
    torch.cuda.synchronize()
    sets.check()
    g_off, g_ids, g_crho = parity.gpu_sets_to_host(sets, 0, h * w)
    assert orc.offsets[-1] > 5 * h * w          # depth-agnostic sets: several samples per pixel
    st = parity.compare_frustum(orc, g_off, g_ids, g_crho, dep[f].reshape(-1)[orc.pixels])
    assert st["members_checked"] > 0.95 * orc.offsets[-1]
    print(st)


def test_frustum_sets_filter_like_the_oracle(case):
    wl, clip, staged, col, dep, f, orc = case
    sg = _sg()
    h, w = clip.height, clip.width
    sets = sg.scene_gather_frustum(staged, f, sg.FrustumParams(window=wl.window))
    out = sg.scene_filter(staged, sets, sg.FilterParams(sigma_d=0.01)).cpu().numpy().reshape(-1, 3)
    c_ref = col[f].reshape(-1, 3)[orc.pixels]
    dj = (orc.ids.astype(np.int64) >> 22) - wl.window
    want = ofilters.weighted_mean(orc.offsets, orc.colour, orc.rho, dj, c_ref, 0.01)
    # pixels with a member near their own depth (|rho| < 0.1): their weights cannot
    # all vanish on either side. (A pixel below the near plane, depth 0.005 in the
    # ragged clip, has lost its own sample; every member's depth Gaussian underflows,
    # to 0 / 0 on both sides.)
    seg = np.repeat(np.arange(orc.offsets.size - 1), np.diff(orc.offsets))
    close = np.zeros(orc.offsets.size - 1, dtype=bool)
    close[seg[np.abs(orc.rho) < 0.1]] = True
    keep = ~_unsure(orc) & close
    assert keep.mean() > 0.7
    got = out[keep].astype(np.float64)
    assert np.isfinite(got).all()
    err = np.abs(got - want[keep]).max()
    assert err <= parity.COLOUR_TOL, err


def test_frustum_capacity_overflow_flag_and_no_overrun():
    wl, clip, staged, col, dep, f, orc = _case("small")
    sg = _sg()
    prm = sg.FrustumParams(window=wl.window)
    exact = sg.scene_gather_frustum(staged, f, prm)
    total = exact.total()
    cap = total // 2
    big = sg.alloc_sets(staged, f, f + 1, wl.window, total)
    big.ids.fill_(-7)
    ws = torch.empty(sg.scene_frustum_workspace_size(staged, f, prm), dtype=torch.uint8, device="cuda")
    short = sg.SampleSets(f, f + 1, wl.window, big.offsets, big.ids[:cap], big.crho[:cap], big.status)
    import ctypes
    cc, pp = staged.c_struct(), prm.c_struct()
    lib = sg._lib
    ss = short.c_struct()
    assert lib.scene_frustum_count(ctypes.byref(cc), f, ctypes.byref(pp), ctypes.byref(ss), ws.data_ptr(),
                                   ws.numel(), None) == 0
    assert lib.scene_frustum_scatter(ctypes.byref(cc), f, ctypes.byref(pp), ctypes.byref(ss), ws.data_ptr(),
                                     ws.numel(), None) == 0
    torch.cuda.synchronize()
    assert short.flags() & sg.SG_FLAG_CAPACITY
    assert bool((big.ids[cap:] == -7).all())
    off = big.offsets.cpu().numpy()
    last = int(off[1:][off[1:] <= cap].max())
    assert torch.equal(big.ids[:last], exact.ids[:last])
    # the flagged sets object again, now with the whole arena: the count pass
    # clears the status word, so no stale flag of the earlier call survives
    full = big.c_struct()
    assert lib.scene_frustum_count(ctypes.byref(cc), f, ctypes.byref(pp), ctypes.byref(full), ws.data_ptr(),
                                   ws.numel(), None) == 0
    assert lib.scene_frustum_scatter(ctypes.byref(cc), f, ctypes.byref(pp), ctypes.byref(full), ws.data_ptr(),
                                     ws.numel(), None) == 0
    torch.cuda.synchronize()
    assert big.flags() == 0
    assert torch.equal(big.ids[:total], exact.ids[:total])


def _reach_per_tile(dep_j, c2w_j, c2w_f, fx, fy, cx, cy, rb=2, tile=16):
    """Points of frame J carried into f's view (float64), filed under their nearest
    output pixel: the records within a tile's reach (tile + 2 rb buckets square)."""
    h, w = dep_j.shape
    yy, xx = np.mgrid[0:h, 0:w]
    d = dep_j.astype(np.float64)
    xc = np.stack([d * (xx - cx) / fx, d * (yy - cy) / fy, d], -1).reshape(-1, 3)
    xf = (xc @ c2w_j[:3, :3].T + c2w_j[:3, 3] - c2w_f[:3, 3]) @ c2w_f[:3, :3]
    with np.errstate(invalid="ignore", divide="ignore"):
        u, v = fx * xf[:, 0] / xf[:, 2] + cx, fy * xf[:, 1] / xf[:, 2] + cy
        ok = np.isfinite(u) & np.isfinite(v) & (xf[:, 2] > 0.01)
    bx, by = np.floor(u[ok] + 0.5).astype(np.int64), np.floor(v[ok] + 0.5).astype(np.int64)
    keep = (bx >= -rb) & (bx < w + rb) & (by >= -rb) & (by < h + rb)
    grid = np.zeros((h + 2 * rb, w + 2 * rb), np.int64)
    np.add.at(grid, (by[keep] + rb, bx[keep] + rb), 1)
    return [int(grid[ty:ty + tile + 2 * rb, tx:tx + tile + 2 * rb].sum())
            for ty in range(0, h, tile) for tx in range(0, w, tile)]


def test_frustum_dense_frame_matches_oracle():
    """A window frame whose camera sits 8 m in front of the output camera: its points
    land at z' ~ d + 8 and crowd up to ~24 to an output bucket, so some tiles' reachable
    records outgrow the 768 the count and scatter stage in LDS (those read the frame
    from global memory) and some (p, J) pairs hold more members than the 16 the
    per-thread sort takes (emitted by repeated minimum); the sets must still equal the
    oracle's."""
    sg = _sg()
    wl = configs.tiny(seed=4, width=64, height=48, n_frames=3, window=1)
    clip = generate(wl.spec)
    c2w = clip.cam_to_world.clone()
    c2w[0] = c2w[1]
    c2w[0, :3, 3] += 8.0 * c2w[1, :3, 2]
    clip.cam_to_world = c2w
    f = 1
    col = ostaging.colour_q(clip.rgb_u8.cpu().numpy())
    dep = ostaging.depth_q(clip.depth.cpu().numpy())
    reach = _reach_per_tile(dep[0], c2w[0].numpy(), c2w[1].numpy(), clip.fx, clip.fy, clip.cx, clip.cy)
    assert max(reach) > 768 and min(reach) <= 768, reach
    orc = ofr.gather_frustum(col, dep, c2w.numpy(), clip.fx, clip.fy, clip.cx, clip.cy, f,
                             ofr.FrustumParams(window=wl.window))
    seg = np.repeat(np.arange(orc.offsets.size - 1), np.diff(orc.offsets))
    slot0 = (orc.ids.astype(np.int64) >> 22) == 0
    assert np.bincount(seg[slot0], minlength=orc.offsets.size - 1).max() > 16
    staged = _stage(clip)
    sets = sg.scene_gather_frustum(staged, f, sg.FrustumParams(window=wl.window))
    torch.cuda.synchronize()
    sets.check()
    h, w = clip.height, clip.width
    g_off, g_ids, g_crho = parity.gpu_sets_to_host(sets, 0, h * w)
    st = parity.compare_frustum(orc, g_off, g_ids, g_crho, dep[f].reshape(-1)[orc.pixels])
    assert st["members_checked"] > 0.95 * orc.offsets[-1]
    print(st, "tile reach", reach)


def test_frustum_in_place_arena_matches_fresh_sets():
    """scene_gather_frustum(sets=...) fills a given arena without allocating or
    synchronising; twice in a row into the same arena it gives the fresh call's sets."""
    wl, clip, staged, col, dep, f, orc = _case("ragged")
    sg = _sg()
    prm = sg.FrustumParams(window=wl.window)
    exact = sg.scene_gather_frustum(staged, f, prm)
    total = exact.total()
    arena = sg.alloc_sets(staged, f, f + 1, wl.window, total + 17)
    ws = torch.empty(sg.scene_frustum_workspace_size(staged, f, prm), dtype=torch.uint8, device="cuda")
    for _ in range(2):
        arena.ids.fill_(-3)
        out = sg.scene_gather_frustum(staged, f, prm, ws=ws, sets=arena)
        assert out is arena
        torch.cuda.synchronize()
        arena.check()
        assert torch.equal(arena.offsets, exact.offsets)
        assert torch.equal(arena.ids[:total], exact.ids[:total])
        # bit patterns: rho is NaN for pixels without a valid depth of their own
        assert torch.equal(arena.crho[:total].view(torch.int16), exact.crho[:total].view(torch.int16))
        assert bool((arena.ids[total:] == -3).all())
    with pytest.raises(ValueError):
        sg.scene_gather_frustum(staged, f + 1, prm, ws=ws, sets=arena)
