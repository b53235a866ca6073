"""Seeded solid texture: improved gradient noise and its fractal sum.

This module synthesises *inputs* only; it holds none of the gathering or
filtering arithmetic.

The noise follows the published "improved noise" construction of
K. Perlin (SIGGRAPH 2002): a doubled 256-entry permutation hashes the eight
lattice corners around a point, each corner contributes the dot product of one
of twelve edge-direction gradients with the offset to the point, and the
corner values are blended with the quintic fade 6t^5 - 15t^4 + 10t^3.
It is written here in vectorised torch so it runs on CPU or GPU tensors.
"""
from __future__ import annotations

import torch


def make_permutation(gen: torch.Generator, device="cpu") -> torch.Tensor:
    """Random permutation of 0..255, repeated twice (512 entries, int64)."""
    p = torch.randperm(256, generator=gen)
    return torch.cat([p, p]).to(device)


def _fade(t: torch.Tensor) -> torch.Tensor:
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _corner(h: torch.Tensor, x: torch.Tensor, y: torch.Tensor, z: torch.Tensor) -> torch.Tensor:
    # The low four hash bits select one of the 12 cube-edge gradients
    # (four of them repeated to fill 16 slots), as in the published method.
    h = h & 15
    a = torch.where(h < 8, x, y)
    b = torch.where(h < 4, y, torch.where((h == 12) | (h == 14), x, z))
    a = torch.where((h & 1) == 0, a, -a)
    b = torch.where((h & 2) == 0, b, -b)
    return a + b


def _lerp(t, a, b):
    return a + t * (b - a)


def noise3(p: torch.Tensor, perm: torch.Tensor) -> torch.Tensor:
    """Gradient noise at points p[..., 3] (float64); result roughly in [-1, 1]."""
    fl = torch.floor(p)
    cell = fl.to(torch.int64) & 255
    fr = p - fl
    x, y, z = fr.unbind(-1)
    ix, iy, iz = cell.unbind(-1)
    u, v, w = _fade(x), _fade(y), _fade(z)
    a = perm[ix] + iy
    aa = perm[a] + iz
    ab = perm[a + 1] + iz
    b = perm[ix + 1] + iy
    ba = perm[b] + iz
    bb = perm[b + 1] + iz
    x1, y1, z1 = x - 1.0, y - 1.0, z - 1.0
    n000 = _corner(perm[aa], x, y, z)
    n100 = _corner(perm[ba], x1, y, z)
    n010 = _corner(perm[ab], x, y1, z)
    n110 = _corner(perm[bb], x1, y1, z)
    n001 = _corner(perm[aa + 1], x, y, z1)
    n101 = _corner(perm[ba + 1], x1, y, z1)
    n011 = _corner(perm[ab + 1], x, y1, z1)
    n111 = _corner(perm[bb + 1], x1, y1, z1)
    lo = _lerp(v, _lerp(u, n000, n100), _lerp(u, n010, n110))
    hi = _lerp(v, _lerp(u, n001, n101), _lerp(u, n011, n111))
    return _lerp(w, lo, hi)


def fbm3(p: torch.Tensor, perm: torch.Tensor, octaves: int = 4, base_freq: float = 1.0) -> torch.Tensor:
    """Fractal sum of `octaves` noise layers, frequency doubling and amplitude halving."""
    out = torch.zeros(p.shape[:-1], dtype=p.dtype, device=p.device)
    freq, amp = base_freq, 1.0
    for _ in range(octaves):
        out = out + amp * noise3(p * freq, perm)
        freq *= 2.0
        amp *= 0.5
    return out
