"""Host-side behaviour that needs no GPU: the benchmark's one-GPU contract and the
binding's refusal of host tensors (no host pointer ever reaches the library)."""
import math
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.fixture(scope="module")
def sg():
    from paper_2102_03011_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2102_03011_amd import build
        build.build()
    import paper_2102_03011_amd as mod
    return mod


def _host_clip(sg, n=3, h=8, w=10):
    a, ar = sg.SG_APRON, sg.SG_APRON_RIGHT
    return sg.StagedClip(torch.zeros((n, h + 2 * a, w + a + ar, 4), dtype=torch.float16),
                         torch.zeros((n, h + 2 * a, w + a + ar), dtype=torch.float16),
                         torch.eye(4, dtype=torch.float64).repeat(n, 1, 1), 50.0, 50.0, 4.5, 3.5)


def _host_sets(sg, f=1, window=1, cap=4, h=8, w=10):
    return sg.SampleSets(f, f + 1, window, torch.zeros(h * w + 1, dtype=torch.int64),
                         torch.zeros(cap, dtype=torch.int32), torch.zeros((cap, 4), dtype=torch.float16),
                         torch.zeros(1, dtype=torch.int32))


def test_bindings_refuse_host_tensors(sg):
    clip, sets = _host_clip(sg), _host_sets(sg)
    calls = [
        lambda: sg.scene_frame_sharpness(clip),
        lambda: sg.scene_filter_frames(clip, sets, sg.FilterParams(sigma_d=0.01), torch.ones(3)),
        lambda: sg.scene_inpaint(clip, sets, torch.zeros((3, 8, 10), dtype=torch.uint8), 0.2),
        lambda: sg.scene_box_mask(clip, (-1, -1, 0), (1, 1, 2)),
        lambda: sg.scene_estimate_depth(clip, 1, 1, torch.ones(4)),
        lambda: sg.scene_gather_frustum(clip, 1, sg.FrustumParams(window=1)),
        lambda: sg.scene_filter(clip, sets, sg.FilterParams(sigma_d=0.01)),
    ]
    for k, call in enumerate(calls):
        with pytest.raises(sg.SceneGatherError, match="GPU tensor"):
            call()


def test_frustum_params_reach_the_library_checks(sg):
    # an invalid frustum size is refused by the library's host checks (before any
    # allocation or GPU work)
    clip = _host_clip(sg)
    for bad in (sg.FrustumParams(window=1, l=0.0), sg.FrustumParams(window=1, l=math.nan),
                sg.FrustumParams(window=-1), sg.FrustumParams(window=1, near=0.0)):
        with pytest.raises(sg.SceneGatherError):
            sg.scene_frustum_workspace_size(clip, 1, bad)
    assert sg.scene_frustum_workspace_size(clip, 1, sg.FrustumParams(window=1)) > 0
