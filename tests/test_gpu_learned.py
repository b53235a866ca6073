"""GPU parity of the learned per-sample weights (inference and training step).

The HIP kernels read the records of a gather; the oracle evaluates features,
MLP, set softmax, loss and backward in float64 on the same records with the
device's stored weights (tests/learned_ref.py).

Tolerances. Inference: filtered colour within 1e-3 of the oracle on the 0-1
scale (the colour contract of the gather/filter path). The kernels carry every
matrix-core operand as a bfloat16 hi/lo pair (about 16 significant bits) and
round no activation to 8 bits, so nothing flips at a rounding boundary: the
logits agree to float32-level error and the colours to about 1e-5. Training:
the gradient accumulates O(1e5) float32 products per parameter (relative error
~1e-5 typical), so each parameter tensor must agree within 5e-3 in relative L2
norm and the loss within 1e-4 relative. The output bias b3 has no gradient at
all (the set softmax ignores a constant shift): it must vanish to float32 noise.
"""
import math

import numpy as np
import pytest
import torch

from oracle import learned
from oracle import staging as ostaging
from scenegen import configs, generate
from tests import learned_ref, parity

pytestmark = pytest.mark.gpu

INFER_TOL = parity.COLOUR_TOL
GRAD_REL_TOL = 5e-3


def _sg():
    import paper_2102_03011_amd as sg
    return sg


def _stage(clip):
    sg = _sg()
    return sg.scene_stage(clip.rgb_u8.cuda().contiguous(), clip.depth.cuda().contiguous(),
                          clip.cam_to_world.cuda().contiguous(), clip.fx, clip.fy, clip.cx, clip.cy)


class Case:
    """A staged clip, one gathered output frame and its host-side records."""

    def __init__(self, wl, clip, f):
        sg = _sg()
        self.wl, self.clip, self.f = wl, clip, f
        self.staged = _stage(clip)
        self.params = sg.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near)
        self.sets = sg.scene_gather(self.staged, f, f + 1, self.params)
        torch.cuda.synchronize()
        self.sets.check()
        h, w = clip.height, clip.width
        self.n = h * w
        self.g_off, self.g_ids, self.g_crho = parity.gpu_sets_to_host(self.sets, 0, self.n)
        self.col = ostaging.colour_q(clip.rgb_u8.cpu().numpy())
        self.dep = ostaging.depth_q(clip.depth.cpu().numpy())
        self.cams = clip.cam_to_world.cpu().numpy()

    def features(self, pixels):
        off, ids, crho = learned_ref.records_subset(self.g_off, self.g_ids, self.g_crho, pixels)
        c = self.clip
        x, col = learned_ref.raw_features(off, ids, crho, pixels, self.f, self.dep, self.cams,
                                          c.fx, c.fy, c.cx, c.cy, self.wl.window, self.wl.radius)
        return off, x, col

    def c_ref(self, pixels):
        return self.col[self.f].reshape(-1, 3)[pixels]


def _device_mlp(m: learned.MLP):
    sg = _sg()
    p = sg.MLPParams.from_arrays(m.w1, m.b1, m.w2, m.b2, m.w3, m.b3, m.mean, 1.0 / m.std)
    return p, learned_ref.oracle_mlp_from_device(p)


def _moments(x):
    mean = x.mean(0)
    std = x.std(0)
    std[std < 1e-12] = 1.0
    return mean, std


@pytest.fixture(scope="module")
def small():
    wl = configs.small_plain()
    return Case(wl, generate(wl.spec), 11)


@pytest.fixture(scope="module")
def small_feats(small):
    pixels = np.arange(small.n)
    off, x, col = small.features(pixels)
    return pixels, off, x, col


def test_learned_filter_full_frame_matches_oracle(small, small_feats):
    sg = _sg()
    pixels, off, x, col = small_feats
    assert x.shape[0] > 1_000_000
    mean, std = _moments(x)
    dev, om = _device_mlp(learned_ref.random_mlp(7, mean, std))
    out = sg.scene_filter_learned(small.staged, small.sets, small.params, dev)
    got = out[0].reshape(-1, 3).cpu().numpy().astype(np.float64)
    want = learned_ref.learned_filter(x, col, off, small.c_ref(pixels), om)
    err = np.abs(got - want).max(axis=1)
    print(f"learned filter: max {err.max():.3g}, p99 {np.quantile(err, 0.99):.3g}, records {x.shape[0]}")
    assert err.max() <= INFER_TOL
    # the learned weights matter: the output is not the set's arithmetic mean
    plain = parity.filter_from_records(off, small.g_ids, small.g_crho, small.c_ref(pixels), small.wl.window,
                                       math.inf)
    assert np.abs(plain - want).max() > 20 * INFER_TOL


def test_zero_output_layer_gives_arithmetic_mean(small, small_feats):
    sg = _sg()
    pixels, off, x, col = small_feats
    mean, std = _moments(x)
    m = learned_ref.random_mlp(8, mean, std)
    m.w3[:] = 0.0
    dev, _ = _device_mlp(m)
    out = sg.scene_filter_learned(small.staged, small.sets, small.params, dev)
    got = out[0].reshape(-1, 3).cpu().numpy().astype(np.float64)
    want = parity.filter_from_records(small.g_off, small.g_ids, small.g_crho, small.c_ref(pixels),
                                      small.wl.window, math.inf)
    assert np.abs(got - want).max() <= parity.FILTER_ARITH_TOL


@pytest.mark.parametrize("feature", range(8))
def test_single_feature_logits(small, small_feats, feature):
    """Logit = a monotone function of one feature: localises a wrong feature."""
    sg = _sg()
    pixels, off, x, col = small_feats
    mean, std = _moments(x)
    m = learned.init_mlp(0, mean, std)
    m.w1[:] = 0.0
    m.w2[:] = 0.0
    m.w3[:] = 0.0
    m.b1[:] = 0.0
    m.b2[:] = 0.0
    m.w1[feature, 0] = 1.0
    m.w2[0, 0] = 1.0
    m.w3[0] = 2.0
    m.b3 = 0.0
    dev, om = _device_mlp(m)
    out = sg.scene_filter_learned(small.staged, small.sets, small.params, dev)
    got = out[0].reshape(-1, 3).cpu().numpy().astype(np.float64)
    want = learned_ref.learned_filter(x, col, off, small.c_ref(pixels), om)
    err = np.abs(got - want).max(axis=1)
    assert err.max() <= INFER_TOL, f"feature {feature}: max {err.max():.3g}"


def test_learned_ragged_invalid_and_empty_sets():
    sg = _sg()
    wl = configs.tiny(seed=9, width=100, height=37, n_frames=7, window=3, pose_rot_deg=1.0, pose_trans_m=0.03)
    clip = generate(wl.spec)
    d = clip.depth.clone()
    g = torch.Generator().manual_seed(5)
    r = torch.rand(d.shape, generator=g)
    d[r < 0.03] = float("nan")
    d[(r >= 0.03) & (r < 0.05)] = 0.0
    d[(r >= 0.05) & (r < 0.06)] = float("inf")
    clip.depth = d
    case = Case(wl, clip, 3)
    pixels = np.arange(case.n)
    off, x, col = case.features(pixels)
    empty = np.diff(off) == 0
    assert empty.sum() > 50
    mean, std = _moments(x)
    dev, om = _device_mlp(learned_ref.random_mlp(11, mean, std))
    out = sg.scene_filter_learned(case.staged, case.sets, case.params, dev)
    got = out[0].reshape(-1, 3).cpu().numpy().astype(np.float64)
    want = learned_ref.learned_filter(x, col, off, case.c_ref(pixels), om)
    assert np.abs(got - want).max() <= INFER_TOL
    assert np.array_equal(got[empty], case.c_ref(pixels)[empty])


def test_learned_multi_frame_call(small):
    """Frames [f0, f1) in one call equal the per-frame calls."""
    sg = _sg()
    p = small.params
    sets = sg.scene_gather(small.staged, 9, 12, p)
    m = learned_ref.random_mlp(3, np.zeros(8), np.ones(8))
    dev, _ = _device_mlp(m)
    out = sg.scene_filter_learned(small.staged, sets, p, dev)
    for k, f in enumerate(range(9, 12)):
        one = sg.scene_gather(small.staged, f, f + 1, p)
        o1 = sg.scene_filter_learned(small.staged, one, p, dev)
        assert torch.equal(out[k], o1[0])


def _train_batch(case, n, seed, with_empty=True):
    rng = np.random.default_rng(seed)
    counts = np.diff(case.g_off)
    nonempty = np.flatnonzero(counts > 0)
    pix = rng.choice(nonempty, size=n, replace=False)
    if with_empty and (counts == 0).any():
        pix[:3] = np.flatnonzero(counts == 0)[:3]
    return pix.astype(np.int64)


def test_train_step_gradient_loss_and_adam(small):
    sg = _sg()
    pixels = _train_batch(small, 512, 0)
    off, x, col = small.features(pixels)
    mean, std = _moments(x)
    dev, om = _device_mlp(learned_ref.random_mlp(21, mean, std))
    clean = small.clip.clean[small.f].reshape(-1, 3).cpu().numpy().astype(np.float64)[pixels]
    state = sg.MLPTrainState(dev)
    master0 = state.master.clone()
    lr = 1e-3
    sg.scene_mlp_train_step(small.staged, small.sets, small.params,
                            torch.tensor(pixels, dtype=torch.int32, device="cuda"),
                            torch.tensor(clean, dtype=torch.float32, device="cuda"), state, lr)
    torch.cuda.synchronize()
    xs = learned.standardise(x, om)
    loss, g, _ = learned.loss_and_grads(xs, col, off, small.c_ref(pixels), clean, om)
    got_loss = float(state.loss.item())
    assert abs(got_loss - loss) <= 1e-4 * loss, (got_loss, loss)
    # first Adam step: m = (1 - beta1) g exactly up to one float32 rounding
    g_gpu = state.adam_m.cpu().numpy().astype(np.float64) / 0.1
    sizes = [("w1", 512), ("w2", 4096), ("w3", 64), ("b1", 64), ("b2", 64), ("b3", 1)]
    pos = 0
    for name, n in sizes:
        got = g_gpu[pos:pos + n]
        want = np.ravel(g[name])
        if name == "b3":
            # softmax shift invariance: dL/db3 = sum_s a_s (c_s - O) . dL/dO = 0
            assert abs(want[0]) < 1e-15 and abs(got[0]) <= 1e-4 * np.abs(g["b1"]).max(), got
            pos += n
            continue
        rel = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-30)
        print(f"grad {name}: rel L2 {rel:.3g}, |g| {np.linalg.norm(want):.3g}")
        assert rel <= GRAD_REL_TOL, (name, rel)
        pos += n
    assert pos == sg.SG_MLP_NPARAM
    # closed-form first step on the masters; gradient cleared; bf16 copy refreshed
    gg = state.adam_m.cpu().numpy().astype(np.float64) / 0.1
    want_master = master0.cpu().numpy() - lr * gg / (np.abs(gg) + 1e-8)
    assert np.allclose(state.master.cpu().numpy(), want_master, rtol=0, atol=lr * 1e-3)
    assert torch.count_nonzero(state.grad).item() == 0
    wb = state.params.w.view(torch.bfloat16).float()
    assert torch.equal(wb, state.master[:sg.SG_MLP_NW].to(torch.bfloat16).float())
    assert torch.equal(state.params.b[:129], state.master[sg.SG_MLP_NW:])
    # standardisation entries are not trained
    assert torch.equal(state.params.b[129:], dev.b[129:])


def test_three_adam_steps_match_the_oracle(small):
    """Three device steps in a row. At each step t: the gradient the device used
    (recovered from its first moments, g_t = (m_t - 0.9 m_{t-1}) / 0.1) matches the
    oracle's backward at the device's current forward copy; the second moments follow
    v_t = 0.999 v_{t-1} + 0.001 g_t^2; and the masters moved by Adam's step with the
    bias corrections of step t, lr (m_t / (1 - 0.9^t)) / (sqrt(v_t / (1 - 0.999^t)) + 1e-8).
    From t = 2 on, both decays and both corrections change the result."""
    sg = _sg()
    pixels = _train_batch(small, 512, 4)
    off, x, col = small.features(pixels)
    mean, std = _moments(x)
    dev, _ = _device_mlp(learned_ref.random_mlp(23, mean, std))
    clean = small.clip.clean[small.f].reshape(-1, 3).cpu().numpy().astype(np.float64)[pixels]
    state = sg.MLPTrainState(dev)
    lr = 1e-3
    idx = torch.tensor(pixels, dtype=torch.int32, device="cuda")
    clean_d = torch.tensor(clean, dtype=torch.float32, device="cuda")
    sizes = [("w1", 512), ("w2", 4096), ("w3", 64), ("b1", 64), ("b2", 64), ("b3", 1)]
    m_prev = np.zeros(sg.SG_MLP_NPARAM)
    v_prev = np.zeros(sg.SG_MLP_NPARAM)
    th_prev = state.master.cpu().numpy().astype(np.float64)
    for t in (1, 2, 3):
        om = learned_ref.oracle_mlp_from_device(state.params)
        _, g, _ = learned.loss_and_grads(learned.standardise(x, om), col, off, small.c_ref(pixels), clean, om)
        sg.scene_mlp_train_step(small.staged, small.sets, small.params, idx, clean_d, state, lr)
        torch.cuda.synchronize()
        assert state.t == t
        m_t = state.adam_m.cpu().numpy().astype(np.float64)
        v_t = state.adam_v.cpu().numpy().astype(np.float64)
        th_t = state.master.cpu().numpy().astype(np.float64)
        g_dev = (m_t - 0.9 * m_prev) / 0.1
        pos = 0
        for name, n in sizes:
            if name != "b3":
                want = np.ravel(g[name])
                rel = np.linalg.norm(g_dev[pos:pos + n] - want) / max(np.linalg.norm(want), 1e-30)
                assert rel <= GRAD_REL_TOL, (t, name, rel)
            pos += n
        want_v = 0.999 * v_prev + 0.001 * g_dev * g_dev
        assert np.all(np.abs(v_t - want_v) <= 1e-4 * want_v + 1e-18), t
        step = lr * (m_t / (1 - 0.9 ** t)) / (np.sqrt(v_t / (1 - 0.999 ** t)) + 1e-8)
        assert np.allclose(th_t, th_prev - step, rtol=0, atol=lr * 1e-4), t
        m_prev, v_prev, th_prev = m_t, v_t, th_t


def test_training_lowers_loss(small):
    sg = _sg()
    pixels = _train_batch(small, 1024, 1, with_empty=False)
    off, x, col = small.features(pixels[:256])
    mean, std = _moments(x)
    dev, _ = _device_mlp(learned.init_mlp(5, mean, std))
    clean = torch.tensor(small.clip.clean[small.f].reshape(-1, 3).numpy()[pixels], dtype=torch.float32,
                         device="cuda")
    idx = torch.tensor(pixels, dtype=torch.int32, device="cuda")
    state = sg.MLPTrainState(dev)
    losses = []
    for _ in range(60):
        sg.scene_mlp_train_step(small.staged, small.sets, small.params, idx, clean, state, 3e-3)
        losses.append(float(state.loss.item()))
    print("loss", losses[0], losses[-1])
    assert all(math.isfinite(v) for v in losses)
    assert losses[-1] < 0.8 * losses[0]


def test_train_step_skips_out_of_range_pixels(small):
    sg = _sg()
    dev, _ = _device_mlp(learned.init_mlp(9))
    state = sg.MLPTrainState(dev)
    master0 = state.master.clone()
    idx = torch.tensor([-1, small.n, small.n + 7], dtype=torch.int32, device="cuda")
    clean = torch.zeros(3, 3, dtype=torch.float32, device="cuda")
    sg.scene_mlp_train_step(small.staged, small.sets, small.params, idx, clean, state, 1e-2)
    torch.cuda.synchronize()
    assert float(state.loss.item()) == 0.0
    assert torch.equal(state.master, master0)
    with pytest.raises(sg.SceneGatherError):
        sg.scene_mlp_train_step(small.staged, small.sets, small.params, idx, clean[:2], state, 1e-2)


def test_feature_moments_match_oracle(small):
    sg = _sg()
    pixels = _train_batch(small, 700, 3)
    off, x, _ = small.features(pixels)
    idx = torch.tensor(pixels, dtype=torch.int32, device="cuda")
    mom = sg.scene_feature_moments(small.staged, small.sets, small.params, idx)
    mom = sg.scene_feature_moments(small.staged, small.sets, small.params, idx[:100], moments=mom)
    got = mom.cpu().numpy()
    x2 = np.concatenate([x, x[:off[100]]])
    assert got[0] == x2.shape[0]
    # float32 features summed in float64: relative 1e-5 of the sum of magnitudes
    assert np.all(np.abs(got[1:9] - x2.sum(0)) <= 1e-5 * np.abs(x2).sum(0) + 1e-12)
    assert np.all(np.abs(got[9:] - (x2 * x2).sum(0)) <= 1e-5 * (x2 * x2).sum(0) + 1e-12)
    # the library's standardisation from those moments: mean and 1 / std (population
    # standard deviation) of the features, written into the parameter block only
    p = sg.MLPParams.from_arrays(np.zeros((8, 64)), np.zeros(64), np.zeros((64, 64)), np.zeros(64), np.zeros(64),
                                 0.25, np.zeros(8), np.ones(8))
    before = p.b.clone()
    sg.scene_mlp_standardise(mom, p)
    b = p.b.cpu().numpy().astype(np.float64)
    assert np.allclose(b[132:140], x2.mean(0), rtol=1e-5, atol=1e-9)
    assert np.allclose(b[140:148], 1.0 / x2.std(0), rtol=1e-5)
    assert torch.equal(p.b[:132], before[:132])
    # no spread (a constant feature) and no records: std taken as 1
    m2 = torch.zeros(17, dtype=torch.float64, device="cuda")
    m2[0], m2[1], m2[9] = 4.0, 8.0, 16.0          # feature 0: four records of value 2
    m2[2], m2[10] = 4.0, 20.0                      # feature 1: mean 1, variance 4
    sg.scene_mlp_standardise(m2, p)
    b = p.b.cpu().numpy().astype(np.float64)
    assert b[132] == 2.0 and b[140] == 1.0 and b[133] == 1.0 and b[141] == 0.5
    assert np.all(b[134:140] == 0.0) and np.all(b[142:148] == 1.0)
    sg.scene_mlp_standardise(torch.zeros(17, dtype=torch.float64, device="cuda"), p)
    b = p.b.cpu().numpy()
    assert np.all(b[132:140] == 0.0) and np.all(b[140:148] == 1.0)


def test_training_driver_runs_and_checkpoint_loads(tmp_path):
    from paper_2102_03011_amd import train
    params, meta = train.train(n_clips=2, frames_per_clip=1, steps_per_frame=5, batch=512, stats_clips=1,
                               log=lambda s: None)
    assert math.isfinite(meta["final_loss"]) and meta["steps"] == 10
    path = str(tmp_path / "w.npz")
    train.save_mlp(path, params, meta)
    back, meta2 = train.load_mlp(path)
    assert torch.equal(back.w, params.w) and torch.equal(back.b, params.b)
    assert meta2["steps"] == 10
