"""GPU tests of the batched persistent path (uneven clips in one step).

Each clip's records (offsets, ids, colours + rho) and filtered colours from the
batch must be bit-identical to that clip's own scene_gather / scene_filter calls
(the per-pixel code and the reduction order are the same), for every launch
configuration the autotuner can pick, in eager launches and in graph replays
with changing frames. One clip is also checked against the float64 oracle.
"""
import math

import numpy as np
import pytest
import torch

from oracle import gather as ogather
from oracle import staging as ostaging
from scenegen import configs, generate
from tests import parity

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2102_03011_amd as sg
    return sg


def _stage(clip):
    sg = _sg()
    return sg.scene_stage(clip.rgb_u8.cuda().contiguous(), clip.depth.cuda().contiguous(),
                          clip.cam_to_world.cuda().contiguous(), clip.fx, clip.fy, clip.cx, clip.cy)


class SmallBatch:
    """Five uneven clips: ragged tile edges, different windows, lengths, output
    frames per step, and filter terms."""

    SHAPES = [  # (seed, width, height, frames, window, n_out)
        (31, 160, 90, 12, 5, 1),
        (32, 200, 120, 20, 8, 2),
        (33, 96, 64, 7, 3, 1),
        (34, 130, 77, 15, 10, 3),
        (35, 320, 180, 24, 6, 1),
    ]

    def __init__(self):
        sg = _sg()
        self.wls, self.clips, self.staged = [], [], []
        for seed, w, h, n, win, _ in self.SHAPES:
            wl = configs.tiny(seed=seed, width=w, height=h, n_frames=n, window=win, pose_rot_deg=0.5,
                              pose_trans_m=0.02)
            clip = generate(wl.spec)
            self.wls.append(wl)
            self.clips.append(clip)
            self.staged.append(_stage(clip))
        self.params = [sg.GatherParams(window=wl.window, radius=1, tol=wl.tol, z_near=wl.z_near) for wl in self.wls]
        self.fparams = [sg.FilterParams(sigma_d=0.01), sg.FilterParams(sigma_d=0.02, sigma_c=40 / 255),
                        sg.FilterParams(sigma_d=0.01, sigma_t=6.0), sg.FilterParams(sigma_d=0.01),
                        sg.FilterParams(sigma_d=0.01, sigma_c=0.1, sigma_t=3.0)]
        self.n_out = [s[5] for s in self.SHAPES]

    def batch(self):
        return _sg().Batch(self.staged, self.params, self.fparams, self.n_out)

    def frames(self, step):
        return [(3 + 5 * step + 2 * c) % (self.SHAPES[c][3] - self.n_out[c] + 1) for c in range(len(self.SHAPES))]


def _solo(sb, c, f0):
    sg = _sg()
    sets = sg.scene_gather(sb.staged[c], f0, f0 + sb.n_out[c], sb.params[c])
    out = sg.scene_filter(sb.staged[c], sets, sb.fparams[c])
    return sets, out


def _compare_clip(b, io, sb, c, solo=None):
    sets, out = solo if solo is not None else _solo(sb, c, b.f0[c])
    b0, b1 = b.bases[c], b.bases[c + 1]
    off = io.offsets[b0:b1 + 1]
    lo, hi = int(off[0].item()), int(off[-1].item())
    assert torch.equal(off - lo, sets.offsets), f"clip {c}: offsets differ"
    assert hi - lo == sets.total()
    assert torch.equal(io.ids[lo:hi], sets.ids[:hi - lo]), f"clip {c}: ids differ"
    assert torch.equal(io.crho[lo:hi].view(torch.int16), sets.crho[:hi - lo].view(torch.int16)), f"clip {c}: crho"
    got = io.out[b0:b1].reshape(out.shape)
    assert torch.equal(got.view(torch.int32), out.view(torch.int32)), f"clip {c}: filtered colours differ"


@pytest.fixture(scope="module")
def small_batch():
    return SmallBatch()


def _run(b, io, f0):
    b.set_frames(f0)
    b.gather(io)
    torch.cuda.synchronize()
    io.check()


@pytest.mark.parametrize("cfg", [(4, 1, 4), (1, 1, 1), (8, 4, 8), (2, 2, 2), (1, 4, 8), (8, 1, 1)])
def test_batched_equals_solo(small_batch, cfg):
    sb = small_batch
    b = sb.batch()
    f0 = sb.frames(0)
    b.set_frames(f0)
    io = b.alloc_io(1)
    total = b.count(io)
    io = b.alloc_io(total)
    b.set_config(*cfg)
    _run(b, io, f0)
    assert int(io.offsets[-1].item()) == total
    for c in range(len(sb.SHAPES)):
        _compare_clip(b, io, sb, c)
    b.close()


def test_graph_replay_with_changing_frames(small_batch):
    sb = small_batch
    sg = _sg()
    b = sb.batch()
    caps = []
    for step in range(3):
        b.set_frames(sb.frames(step))
        caps.append(b.count(b.alloc_io(1)))
    io_g = b.alloc_io(max(caps))
    io_e = b.alloc_io(max(caps))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.set_frames(sb.frames(0))
        b.capture(io_g)
        for step in [0, 1, 2, 1]:
            f0 = sb.frames(step)
            b.set_frames(f0)
            b.gather(io_g)          # graph replay
            stream.synchronize()
            torch.zeros(1 << 20, device="cuda").add_(1.0)   # unrelated eager work between replays
            b.set_frames(f0)
            b.gather(io_e)          # eager launches (other buffers)
            stream.synchronize()
            io_g.check()
            total = int(io_g.offsets[-1].item())    # records past the step's total are unwritten
            assert torch.equal(io_g.offsets, io_e.offsets), step
            assert torch.equal(io_g.ids[:total], io_e.ids[:total]), step
            assert torch.equal(io_g.crho[:total].view(torch.int16), io_e.crho[:total].view(torch.int16)), step
            assert torch.equal(io_g.out.view(torch.int32), io_e.out.view(torch.int32)), step
            for c in range(len(sb.SHAPES)):
                _compare_clip(b, io_g, sb, c)
    b.close()
    assert sg is not None


def test_autotune_and_capacity_flag(small_batch):
    sb = small_batch
    b = sb.batch()
    f0 = sb.frames(1)
    b.set_frames(f0)
    total = b.count(b.alloc_io(1))
    small = b.alloc_io(total // 3)
    with pytest.raises(_sg().SceneGatherError):
        b.autotune(small)                      # the arena cannot hold the step
    io = b.alloc_io(total)
    cfg = b.autotune(io)
    assert cfg[0] in (1, 2, 4, 8) and cfg[1] in (1, 2, 4) and cfg[2] in (1, 2, 4, 8)
    assert b.config() == cfg
    _run(b, io, f0)
    for c in range(len(sb.SHAPES)):
        _compare_clip(b, io, sb, c)
    # an arena too small: flagged, nothing written past it, unfitting sets filter to NaN
    guard = torch.full((small.capacity + 64,), -7, dtype=torch.int32, device="cuda")
    small.ids = guard[:small.capacity]
    b.set_frames(f0)
    b.gather(small)
    torch.cuda.synchronize()
    assert small.flags() & _sg().SG_FLAG_CAPACITY
    assert torch.all(guard[small.capacity:] == -7)
    off = small.offsets[1:]
    over = off > small.capacity
    assert torch.isnan(small.out[over]).all() and not torch.isnan(small.out[~over]).any()
    b.close()


def test_batched_clip_against_oracle(small_batch):
    sb = small_batch
    b = sb.batch()
    f0 = sb.frames(2)
    b.set_frames(f0)
    io = b.alloc_io(b.count(b.alloc_io(1)))
    _run(b, io, f0)
    c = 3
    clip, wl = sb.clips[c], sb.wls[c]
    col = ostaging.colour_q(clip.rgb_u8.numpy())
    dep = ostaging.depth_q(clip.depth.numpy())
    rgbd = sb.staged[c].rgbd_image().cpu().numpy().view(np.uint16)
    oprm = ogather.GatherParams(window=wl.window, radius=1, tol=wl.tol, z_near=wl.z_near)
    n = clip.height * clip.width
    sets = b.clip_sets(io, c)
    for fo in range(sb.n_out[c]):
        f = f0[c] + fo
        off = sets.offsets[fo * n:(fo + 1) * n + 1].cpu().numpy()
        lo, hi = off[0], off[-1]
        g_ids = io.ids[lo:hi].cpu().numpy().view(np.uint32)
        g_crho = io.crho[lo:hi].cpu().numpy().view(np.uint16)
        orc = ogather.gather_frame(col, dep, clip.cam_to_world.numpy(), clip.fx, clip.fy, clip.cx, clip.cy, f, oprm)
        parity.compare_membership(orc, off - lo, g_ids, g_crho, rgbd, f, wl.window)
    b.close()


@pytest.fixture(scope="module")
def full_batch():
    """The 32-clip uneven workload at its real sizes (resolutions 640x360 .. 1920x1080,
    30-150 frames, windows 10-40), one output frame per clip per step."""
    sg = _sg()
    wls = configs.batched_clips()
    staged, clips = [], []
    for wl in wls:
        clip = generate(wl.spec, device="cuda", chunk_rays=1 << 20)
        staged.append(sg.scene_stage(clip.rgb_u8, clip.depth, clip.cam_to_world.cuda(), clip.fx, clip.fy,
                                     clip.cx, clip.cy))
        clips.append((clip.n_frames, clip.width, clip.height))
        del clip
    params = [sg.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near) for wl in wls]
    fparams = [sg.FilterParams(sigma_d=wl.sigma_d) for wl in wls]
    return wls, staged, params, fparams, clips


def test_full_batched_workload_equals_solo(full_batch):
    sg = _sg()
    wls, staged, params, fparams, clips = full_batch
    b = sg.Batch(staged, params, fparams, 1)
    f0 = [n // 2 for n, _, _ in clips]
    b.set_frames(f0)
    total = b.count(b.alloc_io(1))
    io = b.alloc_io(total)
    cfg = b.autotune(io)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.set_frames(f0)
        b.capture(io)
        b.gather(io)
        stream.synchronize()
    io.check()
    print(f"batched: {len(wls)} clips, {b.total_pixels} output pixels, {total} records, config {cfg}")
    for c in range(len(wls)):
        sets = sg.scene_gather(staged[c], f0[c], f0[c] + 1, params[c])
        out = sg.scene_filter(staged[c], sets, fparams[c])
        b0, b1 = b.bases[c], b.bases[c + 1]
        off = io.offsets[b0:b1 + 1]
        lo, hi = int(off[0].item()), int(off[-1].item())
        assert torch.equal(off - lo, sets.offsets), c
        assert torch.equal(io.ids[lo:hi], sets.ids[:hi - lo]), c
        assert torch.equal(io.crho[lo:hi].view(torch.int16), sets.crho[:hi - lo].view(torch.int16)), c
        assert torch.equal(io.out[b0:b1].view(torch.int32), out.reshape(-1, 3).view(torch.int32)), c
        del sets, out
    b.close()
    assert math.isfinite(total)
