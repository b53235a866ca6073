"""GPU parity: the HIP path through the C ABI against the float64 oracle.

Every test here needs an MI355X and the built library; all inputs are seeded.
"""
import math

import numpy as np
import pytest
import torch

from oracle import filters as ofilters
from oracle import gather as ogather
from oracle import staging as ostaging
from scenegen import configs, generate

from tests import parity

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2102_03011_amd as sg
    return sg


def _stage(clip, dev="cuda"):
    sg = _sg()
    return sg.scene_stage(clip.rgb_u8.to(dev).contiguous(), clip.depth.to(dev).contiguous(),
                          clip.cam_to_world.to(dev).contiguous(), clip.fx, clip.fy, clip.cx, clip.cy)


def _oracle_planes(clip, staged):
    col = ostaging.colour_q(clip.rgb_u8.cpu().numpy())
    dep = ostaging.depth_q(clip.depth.cpu().numpy())
    rgbd = staged.rgbd_image().cpu().numpy().view(np.uint16)
    return col, dep, rgbd


@pytest.fixture(scope="module")
def small():
    wl = configs.small_plain()
    clip = generate(wl.spec)
    staged = _stage(clip)
    col, dep, rgbd = _oracle_planes(clip, staged)
    return wl, clip, staged, col, dep, rgbd


def _check_frames(wl, clip, staged, col, dep, rgbd, f0, f1, params, fparams=None, pixels=None):
    sg = _sg()
    sets = sg.scene_gather(staged, f0, f1, params)
    torch.cuda.synchronize()
    sets.check()
    fparams = fparams or sg.FilterParams(sigma_d=wl.sigma_d)
    out = sg.scene_filter(staged, sets, fparams).cpu().numpy().astype(np.float64)
    h, w = clip.height, clip.width
    cams = clip.cam_to_world.numpy()
    oprm = ogather.GatherParams(window=params.window, radius=params.radius, tol=params.tol, z_near=params.z_near)
    stats = []
    for fo, f in enumerate(range(f0, f1)):
        g_off, g_ids, g_crho = parity.gpu_sets_to_host(sets, fo, h * w)
        orc = ogather.gather_frame(col, dep, cams, clip.fx, clip.fy, clip.cx, clip.cy, f, oprm, pixels=pixels)
        st = parity.compare_membership(orc, g_off, g_ids, g_crho, rgbd, f, params.window, pixels=pixels)
        pix = orc.pixels
        c_ref = col[f].reshape(-1, 3)[pix]
        # filter arithmetic on the GPU's own records
        if pixels is None:
            rec = parity.filter_from_records(g_off, g_ids, g_crho, c_ref, params.window,
                                             fparams.sigma_d, fparams.sigma_c, fparams.sigma_t)
            got = out[fo].reshape(-1, 3)
            assert np.abs(got - rec).max() <= parity.FILTER_ARITH_TOL
        else:
            got = out[fo].reshape(-1, 3)[pix]
        # end to end against the oracle's own sets (pixels touching a band excluded)
        want = ofilters.filter_sets(orc, col[f], params.window, fparams.sigma_d, fparams.sigma_c, fparams.sigma_t)
        band = parity.pixels_with_band_cases(orc)
        err = np.abs(got - want).max(axis=1)
        assert err[~band].max() <= parity.COLOUR_TOL, f"frame {f}: colour error {err[~band].max():.3g}"
        st["band_pixels"] = int(band.sum())
        st["max_colour_err"] = float(err[~band].max())
        stats.append(st)
    return sets, out, stats


def test_stage_bit_exact(small):
    wl, clip, staged, col, dep, rgbd = small
    # every u8 value and the staged depth round exactly like IEEE binary16 round-to-nearest-even
    assert np.array_equal(parity.f16_to_f64(rgbd[..., :3].copy()), col)
    d_gpu = parity.f16_to_f64(rgbd[..., 3].copy())
    assert np.array_equal(d_gpu, dep)
    assert np.array_equal(staged.depth_image().cpu().numpy().view(np.uint16), rgbd[..., 3])
    # the apron: binary16 NaN depth in both planes, zero colour
    a = sg_apron = _sg().SG_APRON
    full = staged.rgbd.cpu().numpy().view(np.uint16)
    drows = staged.depth_rows().cpu().numpy().view(np.uint16)
    sh = full.shape[1]
    dfull = drows[:, :sh]
    ring = np.ones(full.shape[:3], bool)
    ring[:, a:a + clip.height, a:a + clip.width] = False
    assert full.shape[2] == clip.width + a + _sg().SG_APRON_RIGHT and full.shape[1] == clip.height + 2 * a
    assert sg_apron >= 3 and np.all(dfull[ring] == 0x7E00) and np.all(full[ring][:, 3] == 0x7E00)
    # the depth plane pairs stored rows: an odd row count leaves one more apron row
    assert drows.shape[1] == sh + (sh & 1) and np.all(drows[:, sh:] == 0x7E00)
    assert np.all(full[ring][:, :3] == 0)
    sg = _sg()
    allv = torch.arange(256, dtype=torch.uint8).repeat_interleave(3).reshape(1, 16, 16, 3).cuda()
    d = torch.linspace(0.001, 70000.0, 256, dtype=torch.float32).reshape(1, 16, 16).cuda()
    s = sg.scene_stage(allv, d, torch.eye(4, dtype=torch.float64).reshape(1, 4, 4).cuda(), 1, 1, 0, 0)
    got = s.rgbd_image().cpu().numpy().view(np.uint16)
    want_c = np.arange(256, dtype=np.float64)[:, None].repeat(3, 1) / 255.0
    assert np.array_equal(got[..., :3].reshape(256, 3), want_c.astype(np.float16).view(np.uint16))
    want_d = ostaging.depth_q(d.cpu().numpy()).astype(np.float16).view(np.uint16)
    assert np.array_equal(got[..., 3], want_d)
    # an odd number of stored rows: the row-paired depth plane holds every stored row
    # (equal to the depth channel) and one more apron row
    s2 = sg.scene_stage(allv[:, :15].contiguous(), d[:, :15].contiguous(),
                        torch.eye(4, dtype=torch.float64).reshape(1, 4, 4).cuda(), 1, 1, 0, 0)
    r2 = s2.depth_rows().cpu().numpy().view(np.uint16)
    c2 = s2.rgbd.cpu().numpy().view(np.uint16)[..., 3]
    assert c2.shape[1] % 2 == 1 and r2.shape[1] == c2.shape[1] + 1
    assert np.array_equal(r2[:, :-1], c2) and np.all(r2[:, -1] == 0x7E00)


@pytest.mark.parametrize("f", list(range(24)))
def test_small_workload_frames(small, f):
    """Every output frame of the 320x180, 24-frame workload (window = all frames)."""
    wl, clip, staged, col, dep, rgbd = small
    sg = _sg()
    params = sg.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near)
    _, _, stats = _check_frames(wl, clip, staged, col, dep, rgbd, f, f + 1, params)
    assert stats[0]["records"] > 1_000_000


def test_small_workload_multi_frame_call_and_paper_preset(small):
    wl, clip, staged, col, dep, rgbd = small
    sg = _sg()
    params = sg.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near)
    fp = sg.FilterParams(sigma_d=0.01, sigma_c=40.0 / 255.0, sigma_t=6.0)
    _check_frames(wl, clip, staged, col, dep, rgbd, 6, 9, params, fparams=fp)


@pytest.mark.parametrize("radius,window", [(0, 3), (2, 2), (3, 1)])
def test_radius_and_window_variants(small, radius, window):
    wl, clip, staged, col, dep, rgbd = small
    sg = _sg()
    params = sg.GatherParams(window=window, radius=radius, tol=0.02, z_near=wl.z_near)
    _check_frames(wl, clip, staged, col, dep, rgbd, 1, 3, params)


def test_ragged_tiles_and_invalid_depths():
    # 100 x 37 pixels: neither tile dimension divides the image; invalid depths everywhere
    wl = configs.tiny(seed=9, width=100, height=37, n_frames=7, window=3, pose_rot_deg=1.0, pose_trans_m=0.03)
    clip = generate(wl.spec)
    d = clip.depth.clone()
    g = torch.Generator().manual_seed(5)
    m = torch.rand(d.shape, generator=g)
    d[m < 0.02] = float("nan")
    d[(m >= 0.02) & (m < 0.04)] = 0.0
    d[(m >= 0.04) & (m < 0.05)] = float("inf")
    d[(m >= 0.05) & (m < 0.06)] = -3.0
    d[(m >= 0.06) & (m < 0.07)] = 0.005           # below the near plane
    d[(m >= 0.07) & (m < 0.075)] = 1e6            # binary16 overflow -> inf
    clip.depth = d
    staged = _stage(clip)
    col, dep, rgbd = _oracle_planes(clip, staged)
    sg = _sg()
    params = sg.GatherParams(window=3, radius=1, tol=0.01, z_near=0.01)
    sets, out, _ = _check_frames(wl, clip, staged, col, dep, rgbd, 0, 7, params)
    # empty sets return the stored colour of the output pixel
    off = sets.offsets.cpu().numpy()
    empty = np.diff(off) == 0
    assert empty.sum() > 100
    ref = col.reshape(-1, 3)[empty]
    assert np.array_equal(out.reshape(-1, 3)[empty], ref)


def test_empty_frame_all_invalid():
    wl = configs.tiny(seed=2, width=70, height=9, n_frames=3, window=2)
    clip = generate(wl.spec)
    clip.depth[1] = float("nan")
    staged = _stage(clip)
    sg = _sg()
    params = sg.GatherParams(window=2)
    sets = sg.scene_gather(staged, 1, 2, params)
    out = sg.scene_filter(staged, sets, sg.FilterParams())
    torch.cuda.synchronize()
    assert sets.total() == 0
    want = ostaging.colour_q(clip.rgb_u8[1].numpy()).astype(np.float32)
    assert np.array_equal(out[0].cpu().numpy(), want)


def test_capacity_overflow_flag_and_no_overrun(small):
    wl, clip, staged, col, dep, rgbd = small
    sg = _sg()
    params = sg.GatherParams(window=wl.window)
    exact = sg.scene_gather(staged, 4, 5, params)
    total = exact.total()
    cap = total // 2
    big = sg.alloc_sets(staged, 4, 5, wl.window, total)
    big.ids.fill_(-7)
    small_sets = sg.SampleSets(4, 5, wl.window, big.offsets, big.ids[:cap], big.crho[:cap], big.status)
    sg.scene_gather(staged, 4, 5, params, capacity=cap, sets=small_sets)
    torch.cuda.synchronize()
    assert small_sets.flags() & sg.SG_FLAG_CAPACITY
    assert bool((big.ids[cap:] == -7).all())
    with pytest.raises(sg.SceneGatherError):
        small_sets.check()
    # the records that fit are the exact ones
    off = big.offsets.cpu().numpy()
    fit = off[1:] <= cap
    last = int(off[1:][fit].max())
    assert torch.equal(big.ids[:last], exact.ids[:last])


def test_no_sync_path_matches_exact_count(small):
    wl, clip, staged, col, dep, rgbd = small
    sg = _sg()
    params = sg.GatherParams(window=wl.window)
    a = sg.scene_gather(staged, 10, 12, params)
    b = sg.scene_gather(staged, 10, 12, params, capacity=a.total() + 100)
    torch.cuda.synchronize()
    b.check()
    assert torch.equal(a.offsets, b.offsets)
    n = a.total()
    assert torch.equal(a.ids[:n], b.ids[:n]) and torch.equal(a.crho[:n], b.crho[:n])


def test_max_window_ids(small):
    # w = 511 is the id-packing limit; the window is truncated to the clip
    wl, clip, staged, col, dep, rgbd = small
    sg = _sg()
    params = sg.GatherParams(window=511)
    _check_frames(wl, clip, staged, col, dep, rgbd, 20, 21, params,
                  pixels=np.arange(0, clip.width * clip.height, 37))


def test_wide_frame_at_pixel_limit():
    # W * H = 2^22 exactly (4096 x 1024): largest frame the id packing allows
    wl = configs.tiny(seed=3, width=4096, height=1024, n_frames=3, window=1)
    wl.spec.n_static = 4
    clip = generate(wl.spec, device="cuda")
    staged = _stage(clip)
    col, dep, rgbd = _oracle_planes(clip, staged)
    sg = _sg()
    params = sg.GatherParams(window=1)
    rng = np.random.default_rng(0)
    pix = np.sort(rng.choice(4096 * 1024, 3000, replace=False))
    _check_frames(wl, clip, staged, col, dep, rgbd, 1, 2, params, pixels=pix)


# ---------------------------------------------------------------------------
# fused gather + filter (no stored sets)

def _fused_vs_stored(staged, f0, f1, params, fparams):
    sg = _sg()
    sets = sg.scene_gather(staged, f0, f1, params)
    stored = sg.scene_filter(staged, sets, fparams)
    fused = sg.scene_gather_filter(staged, f0, f1, params, fparams)
    torch.cuda.synchronize()
    sets.check()
    a = fused.cpu().numpy().astype(np.float64)
    b = stored.cpu().numpy().astype(np.float64)
    # same members, same weights: only the order of the float32 additions differs
    assert np.isfinite(a).all()
    assert np.abs(a - b).max() <= parity.FILTER_ARITH_TOL, np.abs(a - b).max()
    empty = (np.diff(sets.offsets.cpu().numpy()) == 0).reshape(a.shape[:3])
    assert np.array_equal(a[empty], b[empty])   # the output pixel's own colour, exactly
    return a, empty


@pytest.mark.parametrize("radius,window,preset", [(1, 23, "depth"), (1, 23, "paper"), (0, 3, "depth"),
                                                   (2, 2, "paper"), (3, 1, "depth")])
def test_fused_gather_filter_equals_stored_path_and_oracle(small, radius, window, preset):
    wl, clip, staged, col, dep, rgbd = small
    sg = _sg()
    params = sg.GatherParams(window=window, radius=radius, tol=wl.tol if radius == 1 else 0.02, z_near=wl.z_near)
    fparams = (sg.FilterParams(sigma_d=0.01) if preset == "depth"
               else sg.FilterParams(sigma_d=0.01, sigma_c=40.0 / 255.0, sigma_t=6.0))
    f0, f1 = 5, 8
    fused, _ = _fused_vs_stored(staged, f0, f1, params, fparams)
    # end to end against the oracle's own sets for one of the frames (band pixels excluded)
    oprm = ogather.GatherParams(window=window, radius=radius, tol=params.tol, z_near=params.z_near)
    f = 6
    orc = ogather.gather_frame(col, dep, clip.cam_to_world.numpy(), clip.fx, clip.fy, clip.cx, clip.cy, f, oprm)
    want = ofilters.filter_sets(orc, col[f], window, fparams.sigma_d, fparams.sigma_c, fparams.sigma_t)
    band = parity.pixels_with_band_cases(orc)
    err = np.abs(fused[f - f0].reshape(-1, 3) - want).max(axis=1)
    assert err[~band].max() <= parity.COLOUR_TOL


def test_fused_gather_filter_ragged_and_invalid_depths():
    wl = configs.tiny(seed=9, width=100, height=37, n_frames=7, window=3, pose_rot_deg=1.0, pose_trans_m=0.03)
    clip = generate(wl.spec)
    d = clip.depth.clone()
    g = torch.Generator().manual_seed(5)
    m = torch.rand(d.shape, generator=g)
    d[m < 0.03] = float("nan")
    d[(m >= 0.03) & (m < 0.05)] = 0.0
    d[(m >= 0.05) & (m < 0.06)] = float("inf")
    d[(m >= 0.06) & (m < 0.07)] = 0.005
    clip.depth = d
    staged = _stage(clip)
    sg = _sg()
    params = sg.GatherParams(window=3, radius=1, tol=0.01, z_near=0.01)
    _, empty = _fused_vs_stored(staged, 0, 7, params, sg.FilterParams(sigma_d=0.01))
    assert empty.sum() > 100
