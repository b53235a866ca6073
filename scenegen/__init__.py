"""Seeded synthetic input generator (scenes, noise models, workloads).

Shared by the oracle tests, the GPU tests and the benchmark; it holds none of
the gathering or filtering arithmetic.
"""
from .scene import Clip, SceneSpec, generate  # noqa: F401
from . import configs  # noqa: F401
