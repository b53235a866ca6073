"""GPU parity of the paper's other filters over stored sets (Sec. 5): the frame
sharpness B(J) and per-frame factors of deblurring (Eq. 5) and computational
shutters (Eq. 10), and masked mean-shift inpainting (Eq. 8-9) with its masks from
a scene-space box, through the C ABI
against the float64 oracle. All inputs are seeded and synthetic.
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

F = 11  # output frame of the small workload (24 frames, window +-23)


def _sg():
    import paper_2102_03011_amd as sg
    return sg


def _stage(clip):
    sg = _sg()
    return sg.scene_stage(clip.rgb_u8.to("cuda").contiguous(), clip.depth.to("cuda").contiguous(),
                          clip.cam_to_world.to("cuda").contiguous(), clip.fx, clip.fy, clip.cx, clip.cy)


def _moving_box_mask(n, h, w, x0, y0, bw, bh, dx):
    """M^J: a bw x bh box at (x0 + dx J, y0) in frame J (clipped to the image)."""
    m = np.zeros((n, h, w), dtype=np.uint8)
    for j in range(n):
        xa = max(0, min(w, x0 + dx * j))
        m[j, y0:y0 + bh, xa:min(w, xa + bw)] = 1
    return m


def _case(wl, clip, f):
    staged = _stage(clip)
    col = ostaging.colour_q(clip.rgb_u8.cpu().numpy())
    dep = ostaging.depth_q(clip.depth.cpu().numpy())
    sg = _sg()
    params = sg.GatherParams(window=wl.window, tol=wl.tol, z_near=wl.z_near)
    sets = sg.scene_gather(staged, f, f + 1, params)
    torch.cuda.synchronize()
    sets.check()
    oprm = ogather.GatherParams(window=wl.window, radius=1, tol=wl.tol, z_near=wl.z_near)
    orc = ogather.gather_frame(col, dep, clip.cam_to_world.numpy(), clip.fx, clip.fy, clip.cx, clip.cy, f, oprm)
    band = parity.pixels_with_band_cases(orc)
    return staged, col, sets, orc, band


@pytest.fixture(scope="module")
def small():
    wl = configs.small_plain()
    clip = generate(wl.spec)
    return (wl, clip) + _case(wl, clip, F)


@pytest.fixture(scope="module")
def ragged():
    # 100 x 37 (ragged tiles) with invalid depths: NaN, 0, +inf and below z_near
    wl = configs.tiny(seed=9, width=100, height=37, n_frames=7, window=3, pose_rot_deg=1.0, pose_trans_m=0.03)
    clip = generate(wl.spec)
    d = clip.depth.clone()
    m = torch.rand(d.shape, generator=torch.Generator().manual_seed(5))
    d[m < 0.03] = float("nan")
    d[(m >= 0.03) & (m < 0.05)] = 0.0
    d[(m >= 0.05) & (m < 0.06)] = float("inf")
    d[(m >= 0.06) & (m < 0.07)] = 0.005
    clip.depth = d
    return (wl, clip) + _case(wl, clip, 3)


def _err(got, want, band):
    e = np.abs(got.reshape(-1, 3).astype(np.float64) - want).max(axis=1)
    return float(e[~band].max())


def test_frame_sharpness_matches_oracle_and_repeats_bit_for_bit(small, ragged):
    sg = _sg()
    for case in (small, ragged):
        wl, clip, staged, col = case[:4]
        b1 = sg.scene_frame_sharpness(staged)
        b2 = sg.scene_frame_sharpness(staged)
        torch.cuda.synchronize()
        assert torch.equal(b1, b2)
        want = ofilters.frame_sharpness(col)
        got = b1.cpu().numpy().astype(np.float64)
        assert np.all(want > 0)
        np.testing.assert_allclose(got, want, rtol=2e-6)


@pytest.mark.parametrize("preset", ["depth", "paper"])
def test_factor_one_is_the_plain_filter(small, preset):
    wl, clip, staged, col, sets = small[:5]
    sg = _sg()
    fp = (sg.FilterParams(sigma_d=0.01) if preset == "depth"
          else sg.FilterParams(sigma_d=0.01, sigma_c=40.0 / 255.0, sigma_t=6.0))
    ones = torch.ones(clip.n_frames, dtype=torch.float32, device="cuda")
    a = sg.scene_filter_frames(staged, sets, fp, ones)
    b = sg.scene_filter(staged, sets, fp)
    torch.cuda.synchronize()
    assert float((a - b).abs().max()) <= 1e-6


@pytest.mark.parametrize("name", ["small", "ragged"])
def test_deblur_weights_match_oracle(name, request):
    wl, clip, staged, col, sets, orc, band = request.getfixturevalue(name)
    sg = _sg()
    f = orc.frame
    # Eq. 5 with the paper's deblurring sigmas (colour 200 of 255, frame 20) and the depth term;
    # each side weights by its own B(J)
    fp = sg.FilterParams(sigma_d=0.01, sigma_c=200.0 / 255.0, sigma_t=20.0)
    got = sg.scene_filter_frames(staged, sets, fp, sg.scene_frame_sharpness(staged)).cpu().numpy()
    want = ofilters.frame_weighted_mean(orc, col[f], wl.window, ofilters.frame_sharpness(col),
                                        0.01, 200.0 / 255.0, 20.0)
    assert _err(got, want, band) <= parity.COLOUR_TOL


def test_shutter_box_and_all_zero_factors(small):
    wl, clip, staged, col, sets, orc, band = small
    sg = _sg()
    fp = sg.FilterParams(sigma_d=math.inf)
    # a box over frames 5 .. 9 that leaves the output frame itself out: pixels seen
    # only outside it keep their input colour
    xi = np.zeros(clip.n_frames, dtype=np.float32)
    xi[5:10] = 1.0
    got = sg.scene_filter_frames(staged, sets, fp, torch.from_numpy(xi).cuda()).cpu().numpy()
    want = ofilters.frame_weighted_mean(orc, col[F], wl.window, xi.astype(np.float64), math.inf)
    assert _err(got, want, band) <= parity.COLOUR_TOL
    # a decaying tail (trails): xi(J) = 0.7^(F - J) for J <= F
    tail = np.where(np.arange(clip.n_frames) <= F, 0.7 ** (F - np.arange(clip.n_frames)), 0.0)
    got = sg.scene_filter_frames(staged, sets, fp, torch.from_numpy(tail.astype(np.float32)).cuda()).cpu().numpy()
    want = ofilters.frame_weighted_mean(orc, col[F], wl.window, tail.astype(np.float32).astype(np.float64), math.inf)
    assert _err(got, want, band) <= parity.COLOUR_TOL
    # every factor zero: the input colour, exactly
    zero = torch.zeros(clip.n_frames, dtype=torch.float32, device="cuda")
    got = sg.scene_filter_frames(staged, sets, sg.FilterParams(sigma_d=0.01), zero).cpu().numpy()
    assert np.array_equal(got.reshape(-1, 3).astype(np.float64), col[F].reshape(-1, 3))


@pytest.mark.parametrize("name", ["small", "ragged"])
def test_inpaint_matches_oracle(name, request):
    wl, clip, staged, col, sets, orc, band = request.getfixturevalue(name)
    sg = _sg()
    f = orc.frame
    n, h, w = clip.n_frames, clip.height, clip.width
    mask = _moving_box_mask(n, h, w, x0=w // 5, y0=h // 4, bw=w // 3, bh=h // 3, dx=max(1, w // 40))
    sigma = 55.0 / 255.0
    got = sg.scene_inpaint(staged, sets, torch.from_numpy(mask).cuda(), sigma, steps=2).cpu().numpy()
    want = ofilters.inpaint_mean_shift(orc, col[f], wl.window, mask.astype(bool), sigma, steps=2)
    assert _err(got, want, band) <= parity.COLOUR_TOL
    # unmasked output pixels keep their input colour exactly
    keep = mask[f].reshape(-1) == 0
    assert np.array_equal(got.reshape(-1, 3)[keep].astype(np.float64), col[f].reshape(-1, 3)[keep])
    # and the masked region did change where it had unmasked evidence
    assert np.abs(got.reshape(-1, 3)[~keep] - col[f].reshape(-1, 3)[~keep]).max() > 0.01


def test_sets_past_the_arena_and_foreign_ids_give_nan(small):
    wl, clip, staged, col, sets = small[:5]
    sg = _sg()
    n, h, w = clip.n_frames, clip.height, clip.width
    params = sg.GatherParams(window=wl.window, tol=wl.tol, z_near=wl.z_near)
    total = sets.total()
    cap = total // 2
    short = sg.scene_gather(staged, F, F + 1, params, capacity=cap)
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    mask = torch.ones((n, h, w), dtype=torch.uint8, device="cuda")
    a = sg.scene_filter_frames(staged, short, sg.FilterParams(sigma_d=0.01), ones).cpu().numpy().reshape(-1, 3)
    b = sg.scene_inpaint(staged, short, mask, 0.2).cpu().numpy().reshape(-1, 3)
    over = short.offsets.cpu().numpy()[1:] > cap
    assert over.any() and not over.all()
    for out in (a, b):
        assert np.isnan(out[over]).all()
        assert np.isfinite(out[~over]).all()
    # ids decoded with a smaller window than the gather's: a pixel with a record whose
    # source frame falls outside the clip is NaN, the rest finite (bounds-checked lookups)
    w_small = 2
    alias = sg.SampleSets(F, F + 1, w_small, sets.offsets, sets.ids, sets.crho, sets.status)
    c = sg.scene_filter_frames(staged, alias, sg.FilterParams(sigma_d=0.01), ones).cpu().numpy().reshape(-1, 3)
    off = sets.offsets.cpu().numpy()
    j = F - w_small + (sets.ids.cpu().numpy().view(np.uint32) >> 22).astype(np.int64)
    outside = (j < 0) | (j >= n)
    seg = np.repeat(np.arange(off.size - 1), np.diff(off))
    want_nan = np.zeros(off.size - 1, dtype=bool)
    want_nan[seg[outside]] = True
    assert want_nan.any()
    assert np.array_equal(np.isnan(c).any(axis=1), want_nan)


@pytest.mark.parametrize("name", ["small", "ragged"])
def test_box_mask_matches_oracle_and_feeds_inpainting(name, request):
    wl, clip, staged, col, sets, orc, band = request.getfixturevalue(name)
    sg = _sg()
    f = orc.frame
    dep = ostaging.depth_q(clip.depth.cpu().numpy())
    cams = clip.cam_to_world.numpy()
    pts = ofilters.scene_points(np.where(np.isfinite(dep) & (dep > 0), dep, 1.0), cams, clip.fx, clip.fy, clip.cx,
                                clip.cy)
    valid = np.isfinite(dep) & (dep > 0)
    # a box around the middle of the scene points of the output frame
    p = pts[f][valid[f]]
    lo = [float(np.quantile(p[:, k], 0.3)) for k in range(3)]
    hi = [float(np.quantile(p[:, k], 0.7)) for k in range(3)]
    lo[2] = float(p[:, 2].min()) - 1.0
    got = sg.scene_box_mask(staged, lo, hi).cpu().numpy()
    want = ofilters.scene_box_mask(dep, cams, clip.fx, clip.fy, clip.cx, clip.cy, lo, hi)
    # same float64 arithmetic in the same order: equal bits, except where a coordinate
    # lies within 1e-12 of a face (none is expected)
    near = np.zeros(dep.shape, dtype=bool)
    for k in range(3):
        for b in (lo[k], hi[k]):
            near |= valid & (np.abs(pts[..., k] - b) <= 1e-12 * max(1.0, abs(b)))
    assert set(np.unique(got)) <= {0, 1}
    assert np.array_equal(got.astype(bool)[~near], want[~near])
    assert 0 < want[f].mean() < 1
    assert not got[~valid].any()
    # inpainting under the box's masks, each side with its own
    sigma = 55.0 / 255.0
    out = sg.scene_inpaint(staged, sets, torch.from_numpy(got).cuda(), sigma).cpu().numpy()
    ref = ofilters.inpaint_mean_shift(orc, col[f], wl.window, want, sigma)
    if not near.any():
        assert _err(out, ref, band) <= parity.COLOUR_TOL


# ---------------------------------------------------------------------------
# Eq. 4 with its scene-space term (scene_filter_xyz) and semi-transparency

def _scene_side(clip, dep):
    """Side in metres of the cube the paper's scene scale refers to: the largest per-axis
    5 %-95 % range of the scene points of every frame (10 scene units = this many metres)."""
    cams = clip.cam_to_world.numpy()
    valid = np.isfinite(dep) & (dep > 0)
    pts = ofilters.scene_points(np.where(valid, dep, 1.0), cams, clip.fx, clip.fy, clip.cx, clip.cy)[valid]
    return float(max(np.quantile(pts[:, k], 0.95) - np.quantile(pts[:, k], 0.05) for k in range(3)))


def _own_sets(sets, orc_frame, n_pix):
    """The GPU's own records as oracle sets (every output pixel of the frame)."""
    g_off, g_ids, g_crho = parity.gpu_sets_to_host(sets, 0, n_pix)
    return ogather.OracleSets(frame=orc_frame, pixels=np.arange(n_pix, dtype=np.int64), offsets=g_off,
                              ids=g_ids.astype(np.uint32), rho=parity.f16_to_f64(g_crho[:, 3].copy()),
                              colour=parity.f16_to_f64(g_crho[:, :3].copy()),
                              marginal=np.zeros(g_ids.size, dtype=bool),
                              maybe_offsets=np.zeros(n_pix + 1, dtype=np.int64),
                              maybe_ids=np.zeros(0, dtype=np.uint32), maybe_rho=np.zeros(0))


@pytest.mark.parametrize("name,preset", [("small", "xyz"), ("small", "paper"), ("small", "deblur"),
                                          ("ragged", "xyz"), ("ragged", "deblur")])
def test_scene_space_filter_matches_oracle(name, preset, request):
    """Eq. 4 with sigma_xyz: a tight 0.1 m with the depth term; the paper's denoising
    preset (sigma_rgb 40, sigma_xyz 10 scene units, sigma_f 6) and deblurring preset
    (Eq. 5: 200, 10, 20, times B(J)) with the scene scale of the clip. Against the
    oracle on its own sets (outside bands, 1e-3) and on the GPU's own records."""
    wl, clip, staged, col, sets, orc, band = request.getfixturevalue(name)
    sg = _sg()
    f = orc.frame
    dep = ostaging.depth_q(clip.depth.cpu().numpy())
    cams = clip.cam_to_world.numpy()
    side = _scene_side(clip, dep)
    if preset == "xyz":
        sd, sc, st, sx, fw = 0.01, math.inf, math.inf, 0.1, None
    elif preset == "paper":
        sd, sc, st, sx, fw = math.inf, 40.0 / 255.0, 6.0, side, None
    else:
        sd, sc, st, sx, fw = math.inf, 200.0 / 255.0, 20.0, side, sg.scene_frame_sharpness(staged)
    gp = sg.GatherParams(window=wl.window, tol=wl.tol, z_near=wl.z_near)
    got = sg.scene_filter_xyz(staged, sets, gp, sg.FilterParams(sigma_d=sd, sigma_c=sc, sigma_t=st), sx,
                              frame_w=fw).cpu().numpy()
    fw_h = None if fw is None else fw.cpu().numpy().astype(np.float64)
    fw_o = None if fw is None else ofilters.frame_sharpness(col)
    want = ofilters.scene_space_weighted_mean(orc, col[f], dep, cams, clip.fx, clip.fy, clip.cx, clip.cy,
                                              wl.window, sd, sc, sx, st, frame_w=fw_o)
    assert _err(got, want, band) <= parity.COLOUR_TOL
    n_pix = clip.height * clip.width
    own = ofilters.scene_space_weighted_mean(_own_sets(sets, f, n_pix), col[f], dep, cams, clip.fx, clip.fy,
                                             clip.cx, clip.cy, wl.window, sd, sc, sx, st, frame_w=fw_h)
    e = np.abs(got.reshape(-1, 3).astype(np.float64) - own).max()
    assert e <= 1e-4, e
    if name == "ragged":
        # output pixels without a valid stored depth have no reference point
        d = dep[f].reshape(-1)
        nor = ~(np.isfinite(d) & (d > 0))
        assert nor.any()
        assert np.array_equal(got.reshape(-1, 3)[nor].astype(np.float64), col[f].reshape(-1, 3)[nor])


def test_scene_space_filter_without_the_term_is_the_plain_filter(small):
    wl, clip, staged, col, sets = small[:5]
    sg = _sg()
    gp = sg.GatherParams(window=wl.window, tol=wl.tol, z_near=wl.z_near)
    for fp in (sg.FilterParams(sigma_d=0.01), sg.FilterParams(sigma_d=0.01, sigma_c=40.0 / 255.0, sigma_t=6.0)):
        a = sg.scene_filter_xyz(staged, sets, gp, fp, math.inf)
        b = sg.scene_filter(staged, sets, fp)
        torch.cuda.synchronize()
        assert float((a - b).abs().max()) <= 1e-6
    b_j = sg.scene_frame_sharpness(staged)
    fp = sg.FilterParams(sigma_d=math.inf, sigma_c=200.0 / 255.0, sigma_t=20.0)
    a = sg.scene_filter_xyz(staged, sets, gp, fp, math.inf, frame_w=b_j)
    b = sg.scene_filter_frames(staged, sets, fp, b_j)
    torch.cuda.synchronize()
    assert float((a - b).abs().max()) <= 1e-6


@pytest.mark.parametrize("name", ["small", "ragged"])
def test_semi_transparency_matches_oracle(name, request):
    wl, clip, staged, col, sets, orc, band = request.getfixturevalue(name)
    sg = _sg()
    f = orc.frame
    n, h, w = clip.n_frames, clip.height, clip.width
    mask = _moving_box_mask(n, h, w, x0=w // 5, y0=h // 4, bw=w // 3, bh=h // 3, dx=max(1, w // 40))
    m = torch.from_numpy(mask).cuda()
    sigma = 80.0 / 255.0
    got = sg.scene_semi_transparent(staged, sets, m, sigma, sigma, steps=2).cpu().numpy()
    want = ofilters.inpaint_mean_shift(orc, col[f], wl.window, mask.astype(bool), sigma, steps=2, sigma_ref=sigma)
    assert _err(got, want, band) <= parity.COLOUR_TOL
    keep = mask[f].reshape(-1) == 0
    assert np.array_equal(got.reshape(-1, 3)[keep].astype(np.float64), col[f].reshape(-1, 3)[keep])
    # the factor around the input pixel pulls the result toward it, against plain inpainting
    plain = sg.scene_inpaint(staged, sets, m, sigma, steps=2).cpu().numpy().reshape(-1, 3)
    cin = col[f].reshape(-1, 3)
    d_semi = np.abs(got.reshape(-1, 3)[~keep] - cin[~keep]).sum(1)
    d_plain = np.abs(plain[~keep] - cin[~keep]).sum(1)
    assert d_semi.mean() < d_plain.mean()
    # sigma_ref infinite is scene_inpaint, bit for bit
    same = sg.scene_semi_transparent(staged, sets, m, sigma, math.inf, steps=2).cpu().numpy().reshape(-1, 3)
    assert np.array_equal(same, plain)
