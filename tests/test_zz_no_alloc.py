"""The allocation-free gather (scene_gather_noalloc, workspace in the library's
static device scratch) against scene_gather with a caller workspace: identical
offsets, ids and records, on two calls in a row, the second one smaller (fewer
output frames, a narrower window), so stale scratch contents of the first call
would show."""
import numpy as np
import pytest
import torch

from scenegen import configs, generate

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2102_03011_amd as sg
    return sg


@pytest.fixture(scope="module")
def staged():
    sg = _sg()
    wl = configs.small_plain()
    clip = generate(wl.spec)
    dev = "cuda"
    return sg.scene_stage(clip.rgb_u8.to(dev).contiguous(), clip.depth.to(dev).contiguous(),
                          clip.cam_to_world.to(dev).contiguous(), clip.fx, clip.fy, clip.cx, clip.cy)


def _same_sets(a, b):
    off_a, off_b = a.offsets.cpu().numpy(), b.offsets.cpu().numpy()
    assert np.array_equal(off_a, off_b)
    n = int(off_a[-1])
    assert np.array_equal(a.ids[:n].cpu().numpy(), b.ids[:n].cpu().numpy())
    assert np.array_equal(a.crho[:n].cpu().numpy().view(np.uint16), b.crho[:n].cpu().numpy().view(np.uint16))


@pytest.mark.parametrize("calls", [[(3, 7, 23, 1), (10, 11, 5, 1)], [(0, 2, 11, 2), (23, 24, 3, 0)]])
def test_noalloc_matches_scene_gather_twice(staged, calls):
    sg = _sg()
    for f0, f1, w, r in calls:
        params = sg.GatherParams(window=w, radius=r)
        want = sg.scene_gather(staged, f0, f1, params)
        torch.cuda.synchronize()
        want.check()
        got = sg.alloc_sets(staged, f0, f1, w, want.capacity)
        # poison the caller's buffers so every value compared is written by the call
        got.offsets.fill_(-7)
        got.ids.fill_(-7)
        got.crho.fill_(float("nan"))
        got.status.fill_(0x55)
        sg.scene_gather_noalloc(staged, f0, f1, params, got)
        torch.cuda.synchronize()
        got.check()
        assert got.flags() == 0
        _same_sets(want, got)


def test_noalloc_flags_a_small_arena(staged):
    """An arena smaller than the step: the capacity flag is set and nothing is
    written past the arena (the records of the pixels that fit equal scene_gather's)."""
    sg = _sg()
    params = sg.GatherParams(window=4)
    want = sg.scene_gather(staged, 5, 6, params)
    torch.cuda.synchronize()
    cap = want.total() // 2
    got = sg.alloc_sets(staged, 5, 6, 4, cap + 64)
    got.ids.fill_(-7)
    sg.scene_gather_noalloc(staged, 5, 6, params, sg.SampleSets(5, 6, 4, got.offsets, got.ids[:cap],
                                                                  got.crho[:cap], got.status))
    torch.cuda.synchronize()
    assert got.flags() & sg.SG_FLAG_CAPACITY
    assert np.array_equal(got.offsets.cpu().numpy(), want.offsets.cpu().numpy())
    assert (got.ids[cap:].cpu().numpy() == -7).all()
