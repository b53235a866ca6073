"""The five synthetic workloads, with their seeds and gather/filter settings.

Names describe the workload; sizes follow the workload descriptions.
Pose noise: 0.2 deg / 1 cm is stated at 320x180 (fx = 300), where it is about
one pixel of reprojection error. At larger resolutions the perturbation is
scaled by 300 / fx so the error stays the same in pixels (the workload text
is silent on pose noise there).
"""
from __future__ import annotations

import random
from dataclasses import dataclass

from .scene import SceneSpec


@dataclass
class Workload:
    name: str
    spec: SceneSpec
    window: int
    radius: int = 1
    tol: float = 0.01
    sigma_d: float = 0.01
    z_near: float = 0.01


def _pose_scaled(width: int):
    s = 320.0 / width
    return 0.2 * s, 0.01 * s


def small_plain(seed: int = 0) -> Workload:
    """320x180, 24 frames, 12 boxes; window = all frames (w = 23)."""
    spec = SceneSpec(width=320, height=180, n_frames=24, n_static=12, n_moving=0, fx=300.0,
                     colour_sigma=8 / 255, depth_noise=0.02, outlier_frac=0.01,
                     pose_rot_deg=0.2, pose_trans_m=0.01, seed=seed)
    return Workload("denoise-320x180-24f-w23", spec, window=23)


def hd_plain(seed: int = 1, n_frames: int = 120) -> Workload:
    """1280x720, 120 frames, 40 static + 3 moving boxes, window +-30."""
    rot, tr = _pose_scaled(1280)
    spec = SceneSpec(width=1280, height=720, n_frames=n_frames, n_static=40, n_moving=3,
                     colour_sigma=8 / 255, depth_noise=0.02, outlier_frac=0.01,
                     pose_rot_deg=rot, pose_trans_m=tr, seed=seed)
    return Workload("denoise-1280x720-120f-w30", spec, window=30)


def full_scale(seed: int = 5, n_frames: int = 300) -> Workload:
    """1920x1080, 300 frames (n_frames: a shorter version), 60 static + 5 moving boxes, window +-50."""
    rot, tr = _pose_scaled(1920)
    spec = SceneSpec(width=1920, height=1080, n_frames=n_frames, n_static=60, n_moving=5,
                     colour_sigma=10 / 255, depth_noise=0.03, outlier_frac=0.02,
                     pose_rot_deg=rot, pose_trans_m=tr, seed=seed)
    return Workload(f"denoise-1920x1080-{n_frames}f-w50", spec, window=50)


def batched_clips(n_clips: int = 32, seed0: int = 100) -> list[Workload]:
    """Uneven clips: resolution, length, noise and window all drawn per clip."""
    out = []
    for i in range(n_clips):
        rng = random.Random(seed0 + i)
        w, h = rng.choice([(640, 360), (960, 540), (1280, 720), (1920, 1080)])
        n = rng.randint(30, 150)
        rot, tr = _pose_scaled(w)
        spec = SceneSpec(width=w, height=h, n_frames=n, n_static=12 + rng.randint(0, 28), n_moving=rng.randint(0, 3),
                         colour_sigma=rng.uniform(4, 12) / 255, depth_noise=rng.uniform(0.01, 0.04),
                         outlier_frac=0.01, pose_rot_deg=rot, pose_trans_m=tr, seed=seed0 + i)
        out.append(Workload(f"clip{i}-{w}x{h}-{n}f", spec, window=rng.randint(10, 40)))
    return out


def learned_train(i: int, held_out: bool = False) -> Workload:
    """640x360 x 60-frame training (seeds 1000+) or held-out (seeds 2000+) clip."""
    rot, tr = _pose_scaled(640)
    seed = (2000 if held_out else 1000) + i
    spec = SceneSpec(width=640, height=360, n_frames=60, n_static=12, n_moving=1,
                     colour_sigma=8 / 255, depth_noise=0.02, outlier_frac=0.01,
                     pose_rot_deg=rot, pose_trans_m=tr, seed=seed)
    return Workload(f"learn-640x360-60f-{seed}", spec, window=30)


def tiny(seed: int = 0, width: int = 16, height: int = 12, n_frames: int = 5, window: int = 4, **kw) -> Workload:
    """A few hundred pixels for all-pairs checks."""
    spec = SceneSpec(width=width, height=height, n_frames=n_frames, n_static=3, n_moving=0,
                     seed=seed, step_m=0.05, **kw)
    return Workload(f"tiny-{width}x{height}-{n_frames}f", spec, window=window)
