"""Python binding of the MI355X scene-space gather + filter library.

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the gather and filter runs in the HIP
kernels of libscenegather.so (see include/scene_gather.h for the contract).
There is no CPU fallback: the library must be built, and every tensor passed
in must live on the GPU.

The functions carry the names of the C entry points they call.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to by soname)

from . import _native


class _Lib:
    """The HIP library, loaded on first use (so the package can be imported to
    build it); a missing library raises ImportError at that first use."""

    def __init__(self):
        self._cdll = None

    def __getattr__(self, name):
        if self._cdll is None:
            self._cdll = _native.load()
        return getattr(self._cdll, name)


_lib = _Lib()

SG_ID_SHIFT = _native.SG_ID_SHIFT
SG_FLAG_CAPACITY = _native.SG_FLAG_CAPACITY
SG_FLAG_INCONSISTENT = _native.SG_FLAG_INCONSISTENT


class SceneGatherError(RuntimeError):
    pass


def _check(status: int, what: str) -> None:
    if status != _native.SG_OK:
        msg = _lib.sg_status_string(int(status)).decode()
        raise SceneGatherError(f"{what}: {msg} (status {status})")


def _stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


def _need_gpu(t: torch.Tensor, name: str, dtype=None) -> None:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise SceneGatherError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise SceneGatherError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise SceneGatherError(f"{name} must be contiguous")


def version() -> int:
    return int(_lib.sg_version())


SG_APRON = _native.SG_APRON
SG_APRON_RIGHT = _native.SG_APRON_RIGHT


@dataclass
class StagedClip:
    """Stored input planes of a clip (all on the GPU), padded by an apron of
    invalid depth and zero colour: SG_APRON rows above and below, SG_APRON
    columns left and SG_APRON_RIGHT columns right of the image."""
    rgbd: torch.Tensor          # [N, H + 2A, W + A + AR, 4] float16: r, g, b (0-1), z-depth
    depth: torch.Tensor         # [N, ceil((H + 2A) / 2), W + A + AR, 2] float16 z-depth, stored
                                # rows paired: [n, P, X, s] is stored row 2P + s, column X
    cam_to_world: torch.Tensor  # [N, 4, 4] float64
    fx: float
    fy: float
    cx: float
    cy: float

    @property
    def num_frames(self) -> int:
        return self.rgbd.shape[0]

    @property
    def height(self) -> int:
        return self.rgbd.shape[1] - 2 * SG_APRON

    @property
    def width(self) -> int:
        return self.rgbd.shape[2] - SG_APRON - SG_APRON_RIGHT

    def rgbd_image(self) -> torch.Tensor:
        """[N, H, W, 4] view of the image pixels (without the apron)."""
        a = SG_APRON
        return self.rgbd[:, a:a + self.height, a:a + self.width, :]

    def depth_rows(self) -> torch.Tensor:
        """[N, 2 ceil((H + 2A) / 2), W + A + AR] copy of the depth planes in stored-row
        order (the apron included; with H odd the last row is an extra apron row)."""
        n, pr, sw, _ = self.depth.shape
        return self.depth.permute(0, 1, 3, 2).reshape(n, 2 * pr, sw)

    def depth_image(self) -> torch.Tensor:
        """[N, H, W] copy of the image pixels' depths."""
        a = SG_APRON
        return self.depth_rows()[:, a:a + self.height, a:a + self.width]

    def c_struct(self) -> _native.SgClip:
        return _native.SgClip(self.width, self.height, self.num_frames, 0,
                              self.rgbd.data_ptr(), self.depth.data_ptr(), self.cam_to_world.data_ptr(),
                              float(self.fx), float(self.fy), float(self.cx), float(self.cy))


@dataclass
class GatherParams:
    window: int
    radius: int = 1
    tol: float = 0.01
    z_near: float = 0.01

    def c_struct(self) -> _native.SgGatherParams:
        return _native.SgGatherParams(int(self.window), int(self.radius), float(self.tol), float(self.z_near))


@dataclass
class SampleSets:
    """CSR sample sets of output frames [f0, f1) (device tensors)."""
    f0: int
    f1: int
    window: int
    offsets: torch.Tensor   # [P + 1] int64
    ids: torch.Tensor       # [capacity] int32 (bit pattern of the uint32 ids)
    crho: torch.Tensor      # [capacity, 4] float16: r, g, b, rho
    status: torch.Tensor    # [1] int32 (bit pattern of the uint32 status word)

    @property
    def capacity(self) -> int:
        return self.ids.shape[0]

    def c_struct(self) -> _native.SgSampleSets:
        return _native.SgSampleSets(self.offsets.data_ptr(), self.ids.data_ptr() if self.capacity else None,
                                    self.crho.data_ptr() if self.capacity else None, int(self.capacity),
                                    self.status.data_ptr())

    def total(self) -> int:
        """Number of records (synchronises with the GPU)."""
        return int(self.offsets[-1].item())

    def flags(self) -> int:
        return int(self.status.item()) & 0xFFFFFFFF

    def check(self) -> None:
        fl = self.flags()
        if fl & SG_FLAG_CAPACITY:
            raise SceneGatherError("sample arena too small (SG_FLAG_CAPACITY)")
        if fl & SG_FLAG_INCONSISTENT:
            raise SceneGatherError("count and scatter passes disagree (SG_FLAG_INCONSISTENT)")


def scene_stage(rgb_u8: torch.Tensor, depth: torch.Tensor, cam_to_world: torch.Tensor,
                fx: float, fy: float, cx: float, cy: float) -> StagedClip:
    """Stage u8 RGB [N,H,W,3] and float32 depth [N,H,W] into binary16 planes."""
    _need_gpu(rgb_u8, "rgb_u8", torch.uint8)
    _need_gpu(depth, "depth", torch.float32)
    _need_gpu(cam_to_world, "cam_to_world", torch.float64)
    n, h, w, c = rgb_u8.shape
    if c != 3 or tuple(depth.shape) != (n, h, w) or tuple(cam_to_world.shape) != (n, 4, 4):
        raise SceneGatherError("shape mismatch between rgb_u8 [N,H,W,3], depth [N,H,W], cam_to_world [N,4,4]")
    a = SG_APRON
    sw = w + a + SG_APRON_RIGHT
    rgbd = torch.empty((n, h + 2 * a, sw, 4), dtype=torch.float16, device=rgb_u8.device)
    d16 = torch.empty((n, (h + 2 * a + 1) // 2, sw, 2), dtype=torch.float16, device=rgb_u8.device)
    _check(_lib.scene_stage(rgb_u8.data_ptr(), depth.data_ptr(), n, w, h, rgbd.data_ptr(), d16.data_ptr(),
                            _stream_handle()), "scene_stage")
    return StagedClip(rgbd, d16, cam_to_world, fx, fy, cx, cy)


def scene_stage_into(clip: StagedClip, rgb_u8: torch.Tensor, depth: torch.Tensor, frame: int) -> None:
    """Re-stage one frame of `clip` in place (streaming use: the frame entering a window)."""
    _need_gpu(rgb_u8, "rgb_u8", torch.uint8)
    _need_gpu(depth, "depth", torch.float32)
    h, w = clip.height, clip.width
    if tuple(rgb_u8.shape) != (h, w, 3) or tuple(depth.shape) != (h, w) or not 0 <= frame < clip.num_frames:
        raise SceneGatherError("scene_stage_into: frame shape or index mismatch")
    _check(_lib.scene_stage(rgb_u8.data_ptr(), depth.data_ptr(), 1, w, h, clip.rgbd[frame].data_ptr(),
                            clip.depth[frame].data_ptr(), _stream_handle()), "scene_stage")


def scene_gather_workspace_size(clip: StagedClip, f0: int, f1: int, params: GatherParams) -> int:
    out = ctypes.c_size_t(0)
    cc, pp = clip.c_struct(), params.c_struct()
    _check(_lib.scene_gather_workspace_size(ctypes.byref(cc), f0, f1, ctypes.byref(pp), ctypes.byref(out)),
           "scene_gather_workspace_size")
    return int(out.value)


def alloc_workspace(clip: StagedClip, f0: int, f1: int, params: GatherParams) -> torch.Tensor:
    nbytes = scene_gather_workspace_size(clip, f0, f1, params)
    return torch.empty(nbytes, dtype=torch.uint8, device=clip.rgbd.device)


def alloc_sets(clip: StagedClip, f0: int, f1: int, window: int, capacity: int) -> SampleSets:
    dev = clip.rgbd.device
    p = (f1 - f0) * clip.height * clip.width
    return SampleSets(f0, f1, window,
                      torch.empty(p + 1, dtype=torch.int64, device=dev),
                      torch.empty(capacity, dtype=torch.int32, device=dev),
                      torch.empty((capacity, 4), dtype=torch.float16, device=dev),
                      torch.zeros(1, dtype=torch.int32, device=dev))


def _call_gather(fn, name, clip, f0, f1, params, sets, ws):
    _need_gpu(ws, "workspace", torch.uint8)
    cc, pp, ss = clip.c_struct(), params.c_struct(), sets.c_struct()
    _check(fn(ctypes.byref(cc), f0, f1, ctypes.byref(pp), ctypes.byref(ss), ws.data_ptr(), ws.numel(),
              _stream_handle()), name)


def scene_gather_count(clip: StagedClip, f0: int, f1: int, params: GatherParams, sets: SampleSets,
                       ws: torch.Tensor) -> None:
    _call_gather(_lib.scene_gather_count, "scene_gather_count", clip, f0, f1, params, sets, ws)


def scene_gather_scatter(clip: StagedClip, f0: int, f1: int, params: GatherParams, sets: SampleSets,
                         ws: torch.Tensor) -> None:
    _call_gather(_lib.scene_gather_scatter, "scene_gather_scatter", clip, f0, f1, params, sets, ws)


def scene_gather(clip: StagedClip, f0: int, f1: int, params: GatherParams, capacity: int | None = None,
                 sets: SampleSets | None = None, ws: torch.Tensor | None = None) -> SampleSets:
    """Gather the sample sets of output frames [f0, f1).

    capacity None: count, synchronise, size the arena exactly, scatter.
    Otherwise the arena holds `capacity` records and the call never synchronises;
    check `sets.check()` afterwards.
    """
    if ws is None:
        ws = alloc_workspace(clip, f0, f1, params)
    if capacity is None:
        tmp = sets if sets is not None else alloc_sets(clip, f0, f1, params.window, 0)
        scene_gather_count(clip, f0, f1, params, tmp, ws)
        total = tmp.total()
        if sets is None or sets.capacity < total:
            sets = alloc_sets(clip, f0, f1, params.window, total)
            sets.offsets.copy_(tmp.offsets)
            sets.status.copy_(tmp.status)
        scene_gather_scatter(clip, f0, f1, params, sets, ws)
        return sets
    if sets is None:
        sets = alloc_sets(clip, f0, f1, params.window, capacity)
    _call_gather(_lib.scene_gather, "scene_gather", clip, f0, f1, params, sets, ws)
    return sets


def scene_gather_noalloc(clip: StagedClip, f0: int, f1: int, params: GatherParams, sets: SampleSets) -> SampleSets:
    """scene_gather into caller-provided sets with the library's static device
    scratch as workspace (no allocation by the library; the caller's `sets` hold
    the arena). Never synchronises; check `sets.check()` afterwards."""
    cc, pp, ss = clip.c_struct(), params.c_struct(), sets.c_struct()
    _check(_lib.scene_gather_noalloc(ctypes.byref(cc), f0, f1, ctypes.byref(pp), ctypes.byref(ss),
                                     _stream_handle()), "scene_gather_noalloc")
    return sets


@dataclass
class FrustumParams:
    """Depth-agnostic frustum gather (include/scene_frustum.h): window +-w, frustum
    side l pixels (the paper's 3), depth range [near, far] (0.01, 1000)."""
    window: int
    l: float = 3.0
    near: float = 0.01
    far: float = 1000.0

    def c_struct(self) -> _native.SgFrustumParams:
        return _native.SgFrustumParams(int(self.window), float(self.l), float(self.near), float(self.far))


def scene_frustum_workspace_size(clip: StagedClip, f: int, params: FrustumParams) -> int:
    out = ctypes.c_size_t(0)
    cc, pp = clip.c_struct(), params.c_struct()
    _check(_lib.scene_frustum_workspace_size(ctypes.byref(cc), f, ctypes.byref(pp), ctypes.byref(out)),
           "scene_frustum_workspace_size")
    return int(out.value)


def scene_gather_frustum(clip: StagedClip, f: int, params: FrustumParams, capacity: int | None = None,
                         ws: torch.Tensor | None = None, sets: SampleSets | None = None) -> SampleSets:
    """Sample sets of output frame f by the depth-agnostic frustum test (every
    observation along each pixel's ray). capacity None: count, synchronise, size
    the arena exactly, scatter; otherwise the arena holds `capacity` records (check
    `sets.check()` afterwards). `sets`: an arena of output frame f to fill in place
    (no allocation, no synchronisation; capacity is then its own)."""
    if ws is None:
        ws = torch.empty(scene_frustum_workspace_size(clip, f, params), dtype=torch.uint8, device=clip.rgbd.device)
    _need_gpu(ws, "workspace", torch.uint8)
    cc, pp = clip.c_struct(), params.c_struct()
    if sets is not None:
        if sets.f0 != f or sets.f1 != f + 1 or sets.window != params.window:
            raise ValueError("sets must hold output frame f with the window of params")
        tmp = sets
    else:
        tmp = alloc_sets(clip, f, f + 1, params.window, 0)
    ts = tmp.c_struct()
    _check(_lib.scene_frustum_count(ctypes.byref(cc), f, ctypes.byref(pp), ctypes.byref(ts), ws.data_ptr(),
                                    ws.numel(), _stream_handle()), "scene_frustum_count")
    if sets is None:
        if capacity is None:
            capacity = tmp.total()
        sets = alloc_sets(clip, f, f + 1, params.window, capacity)
        sets.offsets.copy_(tmp.offsets)
    ss = sets.c_struct()
    _check(_lib.scene_frustum_scatter(ctypes.byref(cc), f, ctypes.byref(pp), ctypes.byref(ss), ws.data_ptr(),
                                      ws.numel(), _stream_handle()), "scene_frustum_scatter")
    return sets


def scene_estimate_depth(clip: StagedClip, f: int, window: int, hypotheses: torch.Tensor,
                         with_cost: bool = True) -> tuple[torch.Tensor, torch.Tensor | None]:
    """Data-term-only depth of frame f over the hypotheses [K] float32 (GPU):
    -> (depth [H, W], least mean patch cost [H, W] or None), float32."""
    _need_gpu(hypotheses, "hypotheses", torch.float32)
    dev = clip.rgbd.device
    nbytes = ctypes.c_size_t(0)
    cc = clip.c_struct()
    _check(_lib.scene_depth_workspace_size(ctypes.byref(cc), f, window, ctypes.byref(nbytes)),
           "scene_depth_workspace_size")
    ws = torch.empty(max(1, int(nbytes.value)), dtype=torch.uint8, device=dev)
    depth = torch.empty((clip.height, clip.width), dtype=torch.float32, device=dev)
    cost = torch.empty_like(depth) if with_cost else None
    _check(_lib.scene_estimate_depth(ctypes.byref(cc), f, window, hypotheses.data_ptr(), int(hypotheses.numel()),
                                     depth.data_ptr(), cost.data_ptr() if cost is not None else None,
                                     ws.data_ptr(), ws.numel(), _stream_handle()), "scene_estimate_depth")
    return depth, cost


@dataclass
class FilterParams:
    sigma_d: float = 0.01
    sigma_c: float = math.inf
    sigma_t: float = math.inf

    def c_struct(self) -> _native.SgFilterParams:
        return _native.SgFilterParams(float(self.sigma_d), float(self.sigma_c), float(self.sigma_t), 0.0)


def scene_filter(clip: StagedClip, sets: SampleSets, params: FilterParams, out: torch.Tensor | None = None) -> torch.Tensor:
    """Weighted mean of each set -> [f1 - f0, H, W, 3] float32."""
    shape = (sets.f1 - sets.f0, clip.height, clip.width, 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=clip.rgbd.device)
    _need_gpu(out, "out", torch.float32)
    if tuple(out.shape) != shape:
        raise SceneGatherError(f"out must have shape {shape}")
    cc, ss, pp = clip.c_struct(), sets.c_struct(), params.c_struct()
    _check(_lib.scene_filter(ctypes.byref(cc), sets.f0, sets.f1, sets.window, ctypes.byref(ss), ctypes.byref(pp),
                             out.data_ptr(), _stream_handle()), "scene_filter")
    return out


def scene_gather_filter(clip: StagedClip, f0: int, f1: int, params: GatherParams, fparams: FilterParams,
                        out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Gather + plain filter in one pass, no stored sets -> [f1 - f0, H, W, 3] float32
    (equal to scene_filter(scene_gather(...)) up to float32 addition order)."""
    shape = (f1 - f0, clip.height, clip.width, 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=clip.rgbd.device)
    _need_gpu(out, "out", torch.float32)
    if tuple(out.shape) != shape:
        raise SceneGatherError(f"out must have shape {shape}")
    if ws is None:
        ws = alloc_workspace(clip, f0, f1, params)
    _need_gpu(ws, "ws")
    cc, pp, fp = clip.c_struct(), params.c_struct(), fparams.c_struct()
    _check(_lib.scene_gather_filter(ctypes.byref(cc), f0, f1, ctypes.byref(pp), ctypes.byref(fp), out.data_ptr(),
                                    ws.data_ptr(), ws.numel() * ws.element_size(), _stream_handle()),
           "scene_gather_filter")
    return out


# ---------------------------------------------------------------------------
# the paper's other filters over the same sets: deblurring, shutters, inpainting

SG_MAX_INPAINT_STEPS = _native.SG_MAX_INPAINT_STEPS


def scene_frame_sharpness(clip: StagedClip, out: torch.Tensor | None = None) -> torch.Tensor:
    """B(J) of the deblurring weight (summed gradient magnitude of each stored
    frame) -> [N] float32."""
    if out is None:
        out = torch.empty((clip.num_frames,), dtype=torch.float32, device=clip.rgbd.device)
    _need_gpu(out, "out", torch.float32)
    if tuple(out.shape) != (clip.num_frames,):
        raise SceneGatherError(f"out must have shape ({clip.num_frames},)")
    cc = clip.c_struct()
    _check(_lib.scene_frame_sharpness(ctypes.byref(cc), out.data_ptr(), _stream_handle()), "scene_frame_sharpness")
    return out


def scene_filter_frames(clip: StagedClip, sets: SampleSets, params: FilterParams, frame_w: torch.Tensor,
                        out: torch.Tensor | None = None) -> torch.Tensor:
    """Weighted mean with a per-source-frame factor frame_w [N] float32 (deblurring:
    scene_frame_sharpness; shutter: xi(J) with every sigma inf) -> [f1 - f0, H, W, 3]."""
    shape = (sets.f1 - sets.f0, clip.height, clip.width, 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=clip.rgbd.device)
    _need_gpu(out, "out", torch.float32)
    _need_gpu(frame_w, "frame_w", torch.float32)
    if tuple(out.shape) != shape:
        raise SceneGatherError(f"out must have shape {shape}")
    if tuple(frame_w.shape) != (clip.num_frames,):
        raise SceneGatherError(f"frame_w must have shape ({clip.num_frames},)")
    cc, ss, pp = clip.c_struct(), sets.c_struct(), params.c_struct()
    _check(_lib.scene_filter_frames(ctypes.byref(cc), sets.f0, sets.f1, sets.window, ctypes.byref(ss),
                                    ctypes.byref(pp), frame_w.data_ptr(), out.data_ptr(), _stream_handle()),
           "scene_filter_frames")
    return out


def scene_inpaint(clip: StagedClip, sets: SampleSets, mask: torch.Tensor, sigma_rgb: float, steps: int = 2,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """Masked mean-shift inpainting; mask [N, H, W] uint8 (nonzero = remove),
    sigma_rgb on the 0..1 colour scale -> [f1 - f0, H, W, 3] float32."""
    shape = (sets.f1 - sets.f0, clip.height, clip.width, 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=clip.rgbd.device)
    _need_gpu(out, "out", torch.float32)
    _need_gpu(mask, "mask", torch.uint8)
    if tuple(out.shape) != shape:
        raise SceneGatherError(f"out must have shape {shape}")
    if tuple(mask.shape) != (clip.num_frames, clip.height, clip.width):
        raise SceneGatherError(f"mask must have shape ({clip.num_frames}, {clip.height}, {clip.width})")
    cc, ss = clip.c_struct(), sets.c_struct()
    _check(_lib.scene_inpaint(ctypes.byref(cc), sets.f0, sets.f1, sets.window, ctypes.byref(ss), mask.data_ptr(),
                              float(sigma_rgb), int(steps), out.data_ptr(), _stream_handle()), "scene_inpaint")
    return out


def scene_semi_transparent(clip: StagedClip, sets: SampleSets, mask: torch.Tensor, sigma_rgb: float,
                           sigma_ref: float, steps: int = 2, out: torch.Tensor | None = None) -> torch.Tensor:
    """Semi-transparency: inpainting whose weights also favour samples coloured like
    the input pixel (Gaussian of sigma_ref around I^f(p)) -> [f1 - f0, H, W, 3] float32."""
    shape = (sets.f1 - sets.f0, clip.height, clip.width, 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=clip.rgbd.device)
    _need_gpu(out, "out", torch.float32)
    _need_gpu(mask, "mask", torch.uint8)
    if tuple(out.shape) != shape:
        raise SceneGatherError(f"out must have shape {shape}")
    if tuple(mask.shape) != (clip.num_frames, clip.height, clip.width):
        raise SceneGatherError(f"mask must have shape ({clip.num_frames}, {clip.height}, {clip.width})")
    cc, ss = clip.c_struct(), sets.c_struct()
    _check(_lib.scene_semi_transparent(ctypes.byref(cc), sets.f0, sets.f1, sets.window, ctypes.byref(ss),
                                       mask.data_ptr(), float(sigma_rgb), float(sigma_ref), int(steps),
                                       out.data_ptr(), _stream_handle()), "scene_semi_transparent")
    return out


def scene_filter_xyz(clip: StagedClip, sets: SampleSets, gparams: GatherParams, params: FilterParams,
                     sigma_xyz: float, frame_w: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """Weighted mean with the full Eq. 4 weight (colour, scene-space position in world
    units, frame time, depth residual) and an optional per-frame factor [N] float32
    (deblurring: scene_frame_sharpness) -> [f1 - f0, H, W, 3] float32."""
    shape = (sets.f1 - sets.f0, clip.height, clip.width, 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=clip.rgbd.device)
    if ws is None:
        ws = alloc_workspace(clip, sets.f0, sets.f1, gparams)
    _need_gpu(out, "out", torch.float32)
    _need_gpu(ws, "workspace", torch.uint8)
    if frame_w is not None:
        _need_gpu(frame_w, "frame_w", torch.float32)
        if tuple(frame_w.shape) != (clip.num_frames,):
            raise SceneGatherError(f"frame_w must have shape ({clip.num_frames},)")
    if tuple(out.shape) != shape:
        raise SceneGatherError(f"out must have shape {shape}")
    cc, ss, pp, gg = clip.c_struct(), sets.c_struct(), params.c_struct(), gparams.c_struct()
    _check(_lib.scene_filter_xyz(ctypes.byref(cc), sets.f0, sets.f1, ctypes.byref(gg), ctypes.byref(ss),
                                 ctypes.byref(pp), float(sigma_xyz),
                                 frame_w.data_ptr() if frame_w is not None else None, ws.data_ptr(), ws.numel(),
                                 out.data_ptr(), _stream_handle()), "scene_filter_xyz")
    return out


def scene_box_mask(clip: StagedClip, lo, hi, out: torch.Tensor | None = None) -> torch.Tensor:
    """Inpainting masks from a world-space box [lo, hi] (3 floats each): 1 where a
    pixel's scene point lies inside -> [N, H, W] uint8."""
    shape = (clip.num_frames, clip.height, clip.width)
    if out is None:
        out = torch.empty(shape, dtype=torch.uint8, device=clip.rgbd.device)
    _need_gpu(out, "out", torch.uint8)
    if tuple(out.shape) != shape:
        raise SceneGatherError(f"out must have shape {shape}")
    box = (ctypes.c_double * 6)(*[float(v) for v in lo], *[float(v) for v in hi])
    cc = clip.c_struct()
    _check(_lib.scene_box_mask(ctypes.byref(cc), box, out.data_ptr(), _stream_handle()), "scene_box_mask")
    return out


# ---------------------------------------------------------------------------
# learned per-sample weights

SG_MLP_NW, SG_MLP_NB, SG_MLP_NPARAM = _native.SG_MLP_NW, _native.SG_MLP_NB, _native.SG_MLP_NPARAM


def _bf16_bits(x: torch.Tensor) -> torch.Tensor:
    return x.to(torch.float32).to(torch.bfloat16).view(torch.int16)


@dataclass
class MLPParams:
    """Device copy of the MLP: w = bfloat16 [W1 (8x64), W2 (64x64), W3 (64)] as int16
    bit patterns, b = float32 [b1 (64), b2 (64), b3, 3 unused, mean (8), 1/std (8)]."""
    w: torch.Tensor
    b: torch.Tensor

    @staticmethod
    def from_arrays(w1, b1, w2, b2, w3, b3, mean, inv_std, device="cuda") -> "MLPParams":
        """Pack the layers (weights rounded to bfloat16) and the standardisation
        (feature mean and 1/std, as the caller gives them) into the device layout."""
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).reshape(-1)
        w = torch.cat([t(w1), t(w2), t(w3)])
        b = torch.cat([t(b1), t(b2), torch.tensor([float(b3), 0.0, 0.0, 0.0], dtype=torch.float64), t(mean),
                       t(inv_std)])
        return MLPParams(_bf16_bits(w).to(device).contiguous(), b.to(torch.float32).to(device).contiguous())

    def c_struct(self) -> _native.SgMlp:
        return _native.SgMlp(self.w.data_ptr(), self.b.data_ptr())

    def weights_f64(self):
        """(w1, b1, w2, b2, w3, b3) as float64 arrays of the stored values."""
        w = self.w.view(torch.bfloat16).to(torch.float64).cpu().numpy()
        b = self.b.to(torch.float64).cpu().numpy()
        return (w[:512].reshape(8, 64), b[:64], w[512:512 + 4096].reshape(64, 64), b[64:128],
                w[512 + 4096:], float(b[128]))


def scene_filter_learned(clip: StagedClip, sets: SampleSets, params: GatherParams, mlp: MLPParams,
                         ws: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Softmax-weighted mean of each set with MLP logits -> [f1 - f0, H, W, 3] float32."""
    shape = (sets.f1 - sets.f0, clip.height, clip.width, 3)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=clip.rgbd.device)
    if ws is None:
        ws = alloc_workspace(clip, sets.f0, sets.f1, params)
    _need_gpu(out, "out", torch.float32)
    _need_gpu(ws, "workspace", torch.uint8)
    _need_gpu(mlp.w, "mlp.w", torch.int16)
    _need_gpu(mlp.b, "mlp.b", torch.float32)
    if tuple(out.shape) != shape or mlp.w.numel() != SG_MLP_NW or mlp.b.numel() != SG_MLP_NB:
        raise SceneGatherError("scene_filter_learned: shape mismatch")
    cc, pp, ss, mm = clip.c_struct(), params.c_struct(), sets.c_struct(), mlp.c_struct()
    _check(_lib.scene_filter_learned(ctypes.byref(cc), sets.f0, sets.f1, ctypes.byref(pp), ctypes.byref(ss),
                                     ctypes.byref(mm), ws.data_ptr(), ws.numel(), out.data_ptr(),
                                     _stream_handle()), "scene_filter_learned")
    return out


class MLPTrainState:
    """Device training state: float32 masters + Adam moments + gradient accumulator,
    the bfloat16 forward copy (`params`) and the last step's loss."""

    def __init__(self, init: MLPParams, w_master=None, b_master=None):
        dev = init.w.device
        if w_master is None:
            w_master = init.w.view(torch.bfloat16).to(torch.float32)
        if b_master is None:
            b_master = init.b[:129].clone()
        self.master = torch.cat([w_master.reshape(-1).to(dev, torch.float32),
                                 b_master.reshape(-1).to(dev, torch.float32)]).contiguous()
        assert self.master.numel() == SG_MLP_NPARAM
        self.adam_m = torch.zeros_like(self.master)
        self.adam_v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.params = MLPParams(init.w.clone(), init.b.clone())
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.t = 0

    def c_struct(self) -> _native.SgMlpTrain:
        return _native.SgMlpTrain(self.master.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr(),
                                  self.grad.data_ptr(), self.params.w.data_ptr(), self.params.b.data_ptr(),
                                  self.loss.data_ptr())


def scene_mlp_train_step(clip: StagedClip, sets: SampleSets, params: GatherParams, pixel_idx: torch.Tensor,
                         clean_rgb: torch.Tensor, state: MLPTrainState, lr: float,
                         ws: torch.Tensor | None = None, t: int | None = None) -> None:
    """One Adam step on the sets of `pixel_idx` (int32, indices into the P pixels of
    [f0, f1)) against clean_rgb [len(pixel_idx), 3] float32, row i the ground truth of
    pixel_idx[i]. Increments state.t unless t is given."""
    _need_gpu(pixel_idx, "pixel_idx", torch.int32)
    _need_gpu(clean_rgb, "clean_rgb", torch.float32)
    if pixel_idx.dim() != 1 or tuple(clean_rgb.shape) != (pixel_idx.numel(), 3):
        raise SceneGatherError("scene_mlp_train_step: pixel_idx must be [n] and clean_rgb [n, 3]")
    if ws is None:
        ws = alloc_workspace(clip, sets.f0, sets.f1, params)
    state.t = state.t + 1 if t is None else t
    cc, pp, ss, st = clip.c_struct(), params.c_struct(), sets.c_struct(), state.c_struct()
    _check(_lib.scene_mlp_train_step(ctypes.byref(cc), sets.f0, sets.f1, ctypes.byref(pp), ctypes.byref(ss),
                                     pixel_idx.data_ptr(), pixel_idx.numel(), clean_rgb.data_ptr(),
                                     ctypes.byref(st), float(lr), int(state.t), ws.data_ptr(), ws.numel(),
                                     _stream_handle()), "scene_mlp_train_step")


N_FEATURES = 8


def scene_feature_moments(clip: StagedClip, sets: SampleSets, params: GatherParams, pixel_idx: torch.Tensor,
                          moments: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Add the record count, per-feature sums and sums of squares over the sets of
    `pixel_idx` into `moments` (float64 [17] on the device; new and zeroed if None)."""
    _need_gpu(pixel_idx, "pixel_idx", torch.int32)
    if moments is None:
        moments = torch.zeros(1 + 2 * N_FEATURES, dtype=torch.float64, device=clip.rgbd.device)
    _need_gpu(moments, "moments", torch.float64)
    if moments.numel() != 1 + 2 * N_FEATURES or pixel_idx.dim() != 1:
        raise SceneGatherError("scene_feature_moments: moments must have 17 entries, pixel_idx be 1-D")
    if ws is None:
        ws = alloc_workspace(clip, sets.f0, sets.f1, params)
    cc, pp, ss = clip.c_struct(), params.c_struct(), sets.c_struct()
    _check(_lib.scene_feature_moments(ctypes.byref(cc), sets.f0, sets.f1, ctypes.byref(pp), ctypes.byref(ss),
                                      pixel_idx.data_ptr(), pixel_idx.numel(), moments.data_ptr(), ws.data_ptr(),
                                      ws.numel(), _stream_handle()), "scene_feature_moments")
    return moments


def scene_mlp_standardise(moments: torch.Tensor, mlp: MLPParams) -> None:
    """Set mlp's feature mean and 1/std from moments accumulated by
    scene_feature_moments (computed on the device)."""
    _need_gpu(moments, "moments", torch.float64)
    _need_gpu(mlp.b, "mlp.b", torch.float32)
    if moments.numel() != 1 + 2 * N_FEATURES or mlp.b.numel() != SG_MLP_NB:
        raise SceneGatherError("scene_mlp_standardise: moments must have 17 entries, mlp.b SG_MLP_NB")
    _check(_lib.scene_mlp_standardise(moments.data_ptr(), mlp.b.data_ptr(), _stream_handle()),
           "scene_mlp_standardise")


# ---------------------------------------------------------------------------
# batched persistent gather + filter over uneven clips


@dataclass
class BatchIO:
    """Device buffers of one batched step (P = total output pixels of the batch)."""
    offsets: torch.Tensor        # [P + 1] int64
    ids: torch.Tensor            # [capacity] int32
    crho: torch.Tensor           # [capacity, 4] float16
    status: torch.Tensor         # [1] int32
    out: torch.Tensor | None     # [P, 3] float32 or None (gather only)

    @property
    def capacity(self) -> int:
        return self.ids.shape[0]

    def c_struct(self) -> _native.SgBatchIo:
        return _native.SgBatchIo(self.offsets.data_ptr(), self.ids.data_ptr() if self.capacity else None,
                                 self.crho.data_ptr() if self.capacity else None, int(self.capacity),
                                 self.status.data_ptr(), self.out.data_ptr() if self.out is not None else None)

    def flags(self) -> int:
        return int(self.status.item()) & 0xFFFFFFFF

    def check(self) -> None:
        fl = self.flags()
        if fl & SG_FLAG_CAPACITY:
            raise SceneGatherError("batch arena too small (SG_FLAG_CAPACITY)")
        if fl & SG_FLAG_INCONSISTENT:
            raise SceneGatherError("count and scatter passes disagree (SG_FLAG_INCONSISTENT)")


class Batch:
    """A planned batch of clips (sg_batch): one CSR over every clip's output pixels,
    persistent count / scan / scatter / filter passes, graph capture, autotuner."""

    def __init__(self, clips, params, fparams, n_out=1):
        n = len(clips)
        if not (len(params) == len(fparams) == n) or n == 0:
            raise SceneGatherError("Batch: clips, params and fparams must have the same non-zero length")
        n_out = [n_out] * n if isinstance(n_out, int) else list(n_out)
        self.clips, self.params, self.fparams, self.n_out = list(clips), list(params), list(fparams), n_out
        self._cc = (_native.SgClip * n)(*[c.c_struct() for c in clips])
        self._pp = (_native.SgGatherParams * n)(*[p.c_struct() for p in params])
        self._ff = (_native.SgFilterParams * n)(*[f.c_struct() for f in fparams])
        self._no = (ctypes.c_int32 * n)(*n_out)
        h = ctypes.c_void_p()
        _check(_lib.sg_batch_create(ctypes.byref(h), self._cc, n, self._pp, self._ff, self._no), "sg_batch_create")
        self._h = h
        self.bases = [int(_lib.sg_batch_pixel_base(h, c)) for c in range(n + 1)]
        self.f0 = None

    @property
    def total_pixels(self) -> int:
        return self.bases[-1]

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.sg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_frames(self, f0) -> None:
        arr = (ctypes.c_int32 * len(self.clips))(*[int(v) for v in f0])
        _check(_lib.sg_batch_set_frames(self._h, arr), "sg_batch_set_frames")
        self.f0 = [int(v) for v in f0]

    def alloc_io(self, capacity: int, with_out: bool = True, device=None) -> BatchIO:
        dev = device or self.clips[0].rgbd.device
        p = self.total_pixels
        return BatchIO(torch.zeros(p + 1, dtype=torch.int64, device=dev),
                       torch.empty(capacity, dtype=torch.int32, device=dev),
                       torch.empty((capacity, 4), dtype=torch.float16, device=dev),
                       torch.zeros(1, dtype=torch.int32, device=dev),
                       torch.empty((p, 3), dtype=torch.float32, device=dev) if with_out else None)

    def count(self, io: BatchIO) -> int:
        """Count pass; returns the step's record total (synchronises)."""
        st = io.c_struct()
        _check(_lib.sg_batch_count(self._h, ctypes.byref(st), _stream_handle()), "sg_batch_count")
        return int(io.offsets[-1].item())

    def gather(self, io: BatchIO) -> None:
        st = io.c_struct()
        _check(_lib.scene_gather_batched(self._h, ctypes.byref(st), _stream_handle()), "scene_gather_batched")

    def capture(self, io: BatchIO) -> None:
        """Capture one step into a graph on torch's current stream (not the null stream)."""
        st = io.c_struct()
        _check(_lib.sg_batch_capture(self._h, ctypes.byref(st), _stream_handle()), "sg_batch_capture")

    def autotune(self, io: BatchIO):
        cfg = (ctypes.c_int32 * 3)()
        st = io.c_struct()
        _check(_lib.sg_batch_autotune(self._h, ctypes.byref(st), _stream_handle(), cfg), "sg_batch_autotune")
        return tuple(cfg)

    def time_passes(self, io: BatchIO) -> dict:
        """One eager step with events between passes -> ms per pass (synchronises)."""
        ms = (ctypes.c_float * 5)()
        st = io.c_struct()
        _check(_lib.sg_batch_time_passes(self._h, ctypes.byref(st), _stream_handle(), ms), "sg_batch_time_passes")
        return dict(zip(("prep", "count", "scan", "scatter", "filter"), list(ms)))

    def set_config(self, th_count: int, k_count: int, th_scatter: int) -> None:
        _check(_lib.sg_batch_set_config(self._h, th_count, k_count, th_scatter), "sg_batch_set_config")

    def config(self):
        cfg = (ctypes.c_int32 * 3)()
        _check(_lib.sg_batch_get_config(self._h, cfg), "sg_batch_get_config")
        return tuple(cfg)

    def clip_sets(self, io: BatchIO, c: int) -> SampleSets:
        """Clip c's sets inside the batch arena (offsets are batch record indices)."""
        b0, b1 = self.bases[c], self.bases[c + 1]
        return SampleSets(self.f0[c], self.f0[c] + self.n_out[c], self.params[c].window, io.offsets[b0:b1 + 1],
                          io.ids, io.crho, io.status)
