"""GPU parity at the full workload sizes, on sampled output pixels.

1920x1080 with a +-50-frame window (300 frames, 60 static + 5 moving boxes) and
1280x720 with +-30 (120 frames, 40 + 3 moving boxes), generated on the GPU from
their seeds. The HIP path runs in the benchmark's launch configuration (one
output frame per call: count, size the arena, scatter, filter); the oracle
computes the sampled pixels one by one. At 1080p the learned-weight filter
(shipped weights) also runs on the same sets and is checked against the float64
oracle on the device's records of the sampled pixels.
"""
import numpy as np
import pytest
import torch

from oracle import depth as odepth
from oracle import filters as ofilters
from oracle import frustum as ofrustum
from oracle import gather as ogather
from oracle import staging as ostaging
from scenegen import configs, generate
from tests import learned_ref, parity

pytestmark = pytest.mark.gpu


def _window_planes(clip, f, w):
    lo, hi = max(0, f - w), min(clip.n_frames - 1, f + w)
    col = ostaging.colour_q(clip.rgb_u8[lo:hi + 1].cpu().numpy())
    dep = ostaging.depth_q(clip.depth[lo:hi + 1].cpu().numpy())
    return lo, col, dep


def _check(wl, clip, staged, f, pixels, report, learned=False):
    import paper_2102_03011_amd as sg
    params = sg.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near)
    sets = sg.scene_gather(staged, f, f + 1, params)
    out = sg.scene_filter(staged, sets, sg.FilterParams(sigma_d=wl.sigma_d))
    torch.cuda.synchronize()
    sets.check()
    h, w = clip.height, clip.width
    g_off, g_ids, g_crho = parity.gpu_sets_to_host(sets, 0, h * w)
    lo, col, dep = _window_planes(clip, f, wl.window)
    cams = clip.cam_to_world[lo:lo + col.shape[0]].numpy()
    oprm = ogather.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near)
    orc = ogather.gather_frame(col, dep, cams, clip.fx, clip.fy, clip.cx, clip.cy, f - lo, oprm, pixels=pixels)
    rgbd = staged.rgbd_image()[lo:lo + col.shape[0]].cpu().numpy().view(np.uint16)
    st = parity.compare_membership(orc, g_off, g_ids, g_crho, rgbd, f - lo, wl.window, pixels=pixels)
    got = out[0].reshape(-1, 3).cpu().numpy().astype(np.float64)[pixels]
    want = ofilters.filter_sets(orc, col[f - lo], wl.window, wl.sigma_d)
    band = parity.pixels_with_band_cases(orc)
    err = np.abs(got - want).max(axis=1)
    assert err[~band].max() <= parity.COLOUR_TOL
    # the fused gather + filter (no stored sets) equals the stored path up to float32 addition order
    fused = sg.scene_gather_filter(staged, f, f + 1, params, sg.FilterParams(sigma_d=wl.sigma_d))
    fused_diff = float((fused[0].double() - out[0].double()).abs().max().item())
    assert fused_diff <= parity.FILTER_ARITH_TOL, fused_diff
    learned_err = None
    if learned:
        from paper_2102_03011_amd import train
        mlp, _ = train.load_mlp()
        lout = sg.scene_filter_learned(staged, sets, params, mlp)
        torch.cuda.synchronize()
        lgot = lout[0].reshape(-1, 3).cpu().numpy().astype(np.float64)[pixels]
        off, ids, crho = learned_ref.records_subset(g_off, g_ids, g_crho, pixels)
        x, lcol = learned_ref.raw_features(off, ids, crho, pixels, f - lo, dep, cams, clip.fx, clip.fy, clip.cx,
                                           clip.cy, wl.window, wl.radius)
        lwant = learned_ref.learned_filter(x, lcol, off, col[f - lo].reshape(-1, 3)[pixels],
                                           learned_ref.oracle_mlp_from_device(mlp))
        learned_err = float(np.abs(lgot - lwant).max())
        assert learned_err <= parity.COLOUR_TOL, learned_err
    # mode F (unquantised inputs): reported, not gated
    colf = ostaging.colour_f(clip.rgb_u8[lo:lo + col.shape[0]].cpu().numpy())
    depf = ostaging.depth_f(clip.depth[lo:lo + col.shape[0]].cpu().numpy())
    orf = ogather.gather_frame(colf, depf, cams, clip.fx, clip.fy, clip.cx, clip.cy, f - lo, oprm, pixels=pixels)
    wantf = ofilters.filter_sets(orf, colf[f - lo], wl.window, wl.sigma_d)
    errf = np.abs(got - wantf).max(axis=1)
    seg_g = np.repeat(np.arange(len(pixels)), np.diff(g_off)[pixels])
    key_g = set(zip(seg_g.tolist(), np.concatenate([g_ids[g_off[p]:g_off[p + 1]] for p in pixels]).tolist()))
    seg_f = np.repeat(np.arange(len(pixels)), np.diff(orf.offsets))
    key_f = set(zip(seg_f.tolist(), orf.ids.tolist()))
    report.append({
        "workload": wl.name, "frame": f, "pixels": len(pixels), **st,
        "band_pixels": int(band.sum()), "max_colour_err_q": float(err[~band].max()),
        "modeF_membership_diff": len(key_g ^ key_f), "modeF_members": len(key_f),
        "modeF_colour_err_max": float(errf.max()), "modeF_colour_err_mean": float(errf.mean()),
        "learned_colour_err_max": learned_err, "fused_vs_stored_max": fused_diff,
    })
    return sets


@pytest.fixture(scope="module")
def report():
    rows = []
    yield rows
    for r in rows:
        print(r)


def _make(wl):
    import paper_2102_03011_amd as sg
    clip = generate(wl.spec, device="cuda", chunk_rays=1 << 20)
    staged = sg.scene_stage(clip.rgb_u8, clip.depth, clip.cam_to_world.cuda(), clip.fx, clip.fy, clip.cx, clip.cy)
    clip.rgb_u8, clip.depth = clip.rgb_u8.cpu(), clip.depth.cpu()
    return wl, clip, staged


@pytest.fixture(scope="module")
def full_clip():
    return _make(configs.full_scale())


@pytest.fixture(scope="module")
def hd_clip():
    return _make(configs.hd_plain())


@pytest.mark.parametrize("f", [0, 150, 299])
def test_full_scale_1080p_w50_sampled(report, full_clip, f):
    wl, clip, staged = full_clip
    rng = np.random.default_rng(f)
    pixels = np.sort(rng.choice(clip.width * clip.height, 2500, replace=False))
    sets = _check(wl, clip, staged, f, pixels, report, learned=True)
    assert sets.total() > (1e8 if f == 150 else 5e7)


@pytest.mark.parametrize("f", [15, 45, 75, 105])
def test_hd_720p_w30_sampled_frames(report, hd_clip, f):
    wl, clip, staged = hd_clip
    rows = np.arange(f % 8, clip.height, 8)
    pixels = (rows[:, None] * clip.width + np.arange(clip.width)[None, :]).ravel()
    _check(wl, clip, staged, f, pixels, report)


def test_full_scale_frustum_w10_sampled(full_clip):
    """Depth-agnostic frustum gather (Sec. 4, Eq. 1-2) at 1920x1080 with a +-10
    window, output frame 72 (the benchmark's frustum leg): 2000 seeded pixels
    against the oracle's definition, computed for those pixels only. Outside the
    oracle's bands: member ids and colours exact, rho within binary16 rounding."""
    import paper_2102_03011_amd as sg
    wl, clip, staged = full_clip
    f, win = 72, 10
    h, w = clip.height, clip.width
    sets = sg.scene_gather_frustum(staged, f, sg.FrustumParams(window=win))
    torch.cuda.synchronize()
    sets.check()
    g_off, g_ids, g_crho = parity.gpu_sets_to_host(sets, 0, h * w)
    pixels = np.sort(np.random.default_rng(72).choice(h * w, 2000, replace=False))
    lo, col, dep = _window_planes(clip, f, win)
    cams = clip.cam_to_world[lo:lo + col.shape[0]].numpy()
    orc = ofrustum.gather_frustum(col, dep, cams, clip.fx, clip.fy, clip.cx, clip.cy, f - lo,
                                  ofrustum.FrustumParams(window=win), pixels=pixels)
    assert orc.offsets[-1] > 20 * pixels.size
    st = parity.compare_frustum(orc, g_off, g_ids, g_crho, dep[f - lo].reshape(-1)[pixels])
    assert st["members_checked"] > 0.95 * orc.offsets[-1]
    print({"frustum_1080p_w10": st})


def test_full_scale_depth_estimate_sampled(full_clip):
    """Data-term depth (Sec. 3) of 1080p frame 72 over +-2 frames and 32 hypotheses
    uniform in inverse depth over 1-30 m (the benchmark's depth leg): 2000 seeded
    pixels against the oracle's cost intervals: the range of each hypothesis's mean
    cost over the roundings float32 may take (projections within the measured
    float32 band of a half-integer)."""
    import paper_2102_03011_amd as sg
    wl, clip, staged = full_clip
    f = 72
    hyp = (1.0 / np.linspace(1.0, 1.0 / 30.0, 32)).astype(np.float32)
    d, cost = sg.scene_estimate_depth(staged, f, 2, torch.from_numpy(hyp).cuda())
    d = d.cpu().numpy().astype(np.float64).reshape(-1)
    cost = cost.cpu().numpy().astype(np.float64).reshape(-1)
    h, w = clip.height, clip.width
    pixels = np.sort(np.random.default_rng(7).choice(h * w, 2000, replace=False))
    lo, col, _ = _window_planes(clip, f, 2)
    cams = clip.cam_to_world[lo:lo + col.shape[0]].numpy()
    lo_c, hi_c = odepth.cost_intervals(col, cams, clip.fx, clip.fy, clip.cx, clip.cy, f - lo, 2,
                                       hyp.astype(np.float64), pixels)
    got, got_cost = d[pixels], cost[pixels]
    # every decision float32 may take: the GPU's hypothesis has a least possible cost
    # no larger than every hypothesis's largest possible one (1e-4 relative for the
    # float32 sums), and the GPU's cost lies in its hypothesis's interval
    exact = 0
    for i in range(pixels.size):
        cand = np.isfinite(lo_c[i])
        if not cand.any():
            assert np.isnan(got[i]) and np.isinf(got_cost[i]), i
            continue
        assert np.isfinite(got[i]), i
        k = int(np.flatnonzero(hyp == np.float32(got[i]))[0])
        assert cand[k], i
        m = np.min(hi_c[i][cand])
        assert lo_c[i, k] <= m * (1 + 1e-4) + 1e-7, (i, k)
        assert lo_c[i, k] * (1 - 1e-4) - 1e-7 <= got_cost[i] <= hi_c[i, k] * (1 + 1e-4) + 1e-7, (i, k)
        exact += int(np.all(lo_c[i][cand] == hi_c[i][cand]))
    assert exact > 0.1 * pixels.size
    print({"depth_1080p_pixels": int(pixels.size), "pixels_without_rounding_ambiguity": exact})
