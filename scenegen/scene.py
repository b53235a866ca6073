"""Seeded synthetic hand-held video clips with known clean radiance.

Stands in for the paper's real hand-held 720p videos (Sec. 6), which are not
available here. Everything is drawn from seeds; nothing here gathers or
filters. The same bytes feed both the oracle and the HIP path.

Conventions (shared by every consumer of a clip):
  * pixel (x, y): x = column, y = row, pixel centres at integer coordinates;
  * pinhole K = [[fx, 0, cx], [0, fy, cy], [0, 0, 1]], cx = (W-1)/2, cy = (H-1)/2;
  * camera frame: x right, y down, z forward; world frame uses the same
    handedness with y pointing down, the ground plane at y = 0 and the
    camera about 1.6 m above it (y = -1.6);
  * poses are camera-to-world 4x4 (row-major), float64;
  * depth is z-depth (distance along the camera's optical axis), not ray length.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from .perlin import fbm3, make_permutation

WALL_Z = 25.0          # back wall plane z = 25 m: every ray hits a surface
GROUND_Y = 0.0         # ground plane (world y points down)
CAMERA_HEIGHT = 1.6


@dataclass
class SceneSpec:
    width: int
    height: int
    n_frames: int
    n_static: int = 12
    n_moving: int = 0
    fx: float | None = None            # default 300 * W / 320 (same field of view)
    colour_sigma: float = 8.0 / 255.0  # Gaussian colour noise on the 0-1 scale
    depth_noise: float = 0.02          # multiplicative Gaussian depth noise (relative)
    outlier_frac: float = 0.01         # fraction of depth pixels replaced by U(2, 20) m
    pose_rot_deg: float = 0.2          # RMS rotation perturbation per frame
    pose_trans_m: float = 0.01         # RMS translation perturbation per frame
    seed: int = 0
    piecewise_constant: bool = False   # one flat colour per object face (no texture)
    static_camera: bool = False        # every frame shares the first camera pose
    step_m: float = 0.03               # camera translation per frame
    rot_step_deg: float = 0.3          # RMS camera rotation per frame

    @property
    def focal(self) -> float:
        return float(self.fx) if self.fx is not None else 300.0 * self.width / 320.0


@dataclass
class Clip:
    spec: SceneSpec
    rgb_u8: torch.Tensor        # [N][H][W][3] uint8, noisy observed colour
    depth: torch.Tensor         # [N][H][W] float32, noisy observed z-depth
    cam_to_world: torch.Tensor  # [N][4][4] float64, perturbed (observed) poses
    fx: float
    fy: float
    cx: float
    cy: float
    clean_u8: torch.Tensor      # [N][H][W][3] uint8, clean radiance quantised like the input
    clean: torch.Tensor         # [N][H][W][3] float32, clean radiance in [0, 1]
    depth_true: torch.Tensor    # [N][H][W] float32
    poses_true: torch.Tensor    # [N][4][4] float64
    face_id: torch.Tensor       # [N][H][W] int32: object * 8 + face
    moving_mask: torch.Tensor   # [N][H][W] bool: pixel sees a moving object
    extra: dict = field(default_factory=dict)

    @property
    def n_frames(self) -> int:
        return self.rgb_u8.shape[0]

    @property
    def height(self) -> int:
        return self.rgb_u8.shape[1]

    @property
    def width(self) -> int:
        return self.rgb_u8.shape[2]


# ----------------------------------------------------------------------------
# small rigid-motion helpers for the *generator* (not used by the method)

def _rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return torch.tensor([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=torch.float64)


def _rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return torch.tensor([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=torch.float64)


def _rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return torch.tensor([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=torch.float64)


def _rodrigues(w: torch.Tensor) -> torch.Tensor:
    th = float(torch.linalg.norm(w))
    if th < 1e-15:
        return torch.eye(3, dtype=torch.float64)
    k = w / th
    kx = torch.tensor([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]], dtype=torch.float64)
    return torch.eye(3, dtype=torch.float64) + math.sin(th) * kx + (1 - math.cos(th)) * (kx @ kx)


def _camera_path(spec: SceneSpec, gen: torch.Generator) -> torch.Tensor:
    """Smooth hand-held random walk: [N][4][4] camera-to-world poses."""
    n = spec.n_frames
    poses = torch.zeros(n, 4, 4, dtype=torch.float64)
    heading = (math.pi / 2) * (1 if torch.rand(1, generator=gen).item() < 0.5 else -1)
    heading += float(torch.empty(1).uniform_(-0.5, 0.5, generator=gen))
    pos = torch.tensor([0.0, -CAMERA_HEIGHT, 0.0], dtype=torch.float64)
    ang = torch.tensor([0.0, math.radians(-10.0), 0.0], dtype=torch.float64)  # yaw, pitch, roll
    ang_mean = ang.clone()
    omega = torch.zeros(3, dtype=torch.float64)
    # AR(1) angular velocity with stationary per-axis RMS = rot_step / sqrt(3)
    rho = 0.8
    s = math.radians(spec.rot_step_deg) / math.sqrt(3.0) * math.sqrt(1 - rho * rho)
    lim = torch.tensor([math.radians(15.0), math.radians(5.0), math.radians(3.0)], dtype=torch.float64)
    hdrift = 0.0
    for i in range(n):
        r = _rot_y(float(ang[0])) @ _rot_x(float(ang[1])) @ _rot_z(float(ang[2]))
        poses[i, :3, :3] = r
        poses[i, :3, 3] = pos
        poses[i, 3, 3] = 1.0
        if spec.static_camera:
            continue
        omega = rho * omega + s * torch.randn(3, generator=gen, dtype=torch.float64)
        ang = ang + omega - 0.05 * (ang - ang_mean)
        ang = torch.maximum(torch.minimum(ang, ang_mean + lim), ang_mean - lim)
        hdrift = 0.9 * hdrift + 0.02 * float(torch.randn(1, generator=gen))
        heading += hdrift
        bob = 0.1 * float(torch.randn(1, generator=gen))
        d = torch.tensor([math.sin(heading), bob, math.cos(heading)], dtype=torch.float64)
        pos = pos + spec.step_m * d / torch.linalg.norm(d)
        pos[1] = 0.98 * pos[1] + 0.02 * (-CAMERA_HEIGHT)
    if spec.static_camera:
        poses[:] = poses[0]
    return poses


def _place_boxes(spec: SceneSpec, path_xz: torch.Tensor, gen: torch.Generator):
    """Axis-aligned boxes resting on the ground, >= 1.5 m from the camera path."""
    n = spec.n_static + spec.n_moving
    los, his, vels = [], [], []
    xmin = float(path_xz[:, 0].min()) - 8.0
    xmax = float(path_xz[:, 0].max()) + 8.0
    zc0 = float(path_xz[:, 1].mean())
    tries = 0
    while len(los) < n:
        tries += 1
        if tries > 100000:
            raise RuntimeError("cannot place boxes")
        u = torch.rand(6, generator=gen, dtype=torch.float64)
        size = 0.3 + 1.7 * u[:3]
        cx = xmin + (xmax - xmin) * float(u[3])
        cz = zc0 + 2.0 + 18.0 * float(u[4])
        moving = len(los) >= spec.n_static
        vel = torch.zeros(3, dtype=torch.float64)
        if moving:
            a = 2 * math.pi * float(u[5])
            sp = 0.01 + 0.02 * float(torch.rand(1, generator=gen))
            vel = torch.tensor([sp * math.cos(a), 0.0, sp * math.sin(a)], dtype=torch.float64)
        lo = torch.tensor([cx - size[0] / 2, GROUND_Y - size[1], cz - size[2] / 2], dtype=torch.float64)
        hi = torch.tensor([cx + size[0] / 2, GROUND_Y, cz + size[2] / 2], dtype=torch.float64)
        # distance (xz) from the path to the box footprint, over the clip
        ok = True
        steps = [0, spec.n_frames - 1] if not moving else range(0, spec.n_frames, max(1, spec.n_frames // 16))
        for k in steps:
            off = vel * k
            dx = torch.clamp(torch.maximum(lo[0] + off[0] - path_xz[:, 0], path_xz[:, 0] - hi[0] - off[0]), min=0)
            dz = torch.clamp(torch.maximum(lo[2] + off[2] - path_xz[:, 1], path_xz[:, 1] - hi[2] - off[2]), min=0)
            if float(torch.sqrt(dx * dx + dz * dz).min()) < 1.5:
                ok = False
                break
        if ok and moving:
            dx = torch.clamp(torch.maximum(lo[0] - path_xz[:, 0], path_xz[:, 0] - hi[0]), min=0)
            dz = torch.clamp(torch.maximum(lo[2] - path_xz[:, 1], path_xz[:, 1] - hi[2]), min=0)
            ok = float(torch.sqrt(dx * dx + dz * dz).min()) >= 1.5
        if not ok:
            continue
        los.append(lo)
        his.append(hi)
        vels.append(vel)
    if n == 0:
        z = torch.zeros(0, 3, dtype=torch.float64)
        return z, z.clone(), z.clone()
    return torch.stack(los), torch.stack(his), torch.stack(vels)


def _raycast(o, rot, dirs_cam, box_lo, box_hi):
    """Nearest hit along rays o + t * (rot @ d). Returns (t, obj, face).

    obj: 0 = ground, 1 = back wall, 2 + i = box i. face in 0..5 for boxes.
    Because d has camera-z component 1, t is the z-depth of the hit.
    """
    d = dirs_cam @ rot.T                       # [R, 3]
    inf = torch.tensor(float("inf"), dtype=d.dtype, device=d.device)
    t_best = torch.where(d[:, 1] > 0, (GROUND_Y - o[1]) / d[:, 1], inf)
    obj = torch.zeros(d.shape[0], dtype=torch.int64, device=d.device)
    face = torch.zeros_like(obj)
    t_wall = torch.where(d[:, 2] > 0, (WALL_Z - o[2]) / d[:, 2], inf)
    m = t_wall < t_best
    t_best = torch.where(m, t_wall, t_best)
    obj = torch.where(m, torch.ones_like(obj), obj)
    nb = box_lo.shape[0]
    if nb:
        with torch.no_grad():
            inv = 1.0 / d                          # [R, 3]
            t1 = (box_lo[None, :, :] - o[None, None, :]) * inv[:, None, :]   # [R, B, 3]
            t2 = (box_hi[None, :, :] - o[None, None, :]) * inv[:, None, :]
            tn = torch.minimum(t1, t2)
            tf = torch.maximum(t1, t2)
            tnear, axis = tn.max(dim=2)            # [R, B]
            tfar = tf.min(dim=2).values
            hit = (tnear <= tfar) & (tnear > 0)
            tnear = torch.where(hit, tnear, inf)
            tb, ib = tnear.min(dim=1)              # [R]
            ax = axis.gather(1, ib[:, None])[:, 0]
            m = tb < t_best
            t_best = torch.where(m, tb, t_best)
            obj = torch.where(m, ib + 2, obj)
            sgn = (d.gather(1, ax[:, None])[:, 0] < 0).to(torch.int64)
            face = torch.where(m, 2 * ax + sgn, face)
    return t_best, obj, face


@dataclass
class SceneSetup:
    """Everything a clip's seed fixes before rendering: camera path (true and
    observed poses), boxes, texture tables and the seed of the observation noise."""
    poses: torch.Tensor       # [N][4][4] true camera-to-world
    noisy: torch.Tensor       # [N][4][4] observed (perturbed) camera-to-world
    box_lo: torch.Tensor
    box_hi: torch.Tensor
    box_vel: torch.Tensor
    perm: torch.Tensor
    base: torch.Tensor
    shift: torch.Tensor
    face_col: torch.Tensor
    moving: torch.Tensor
    noise_seed: int


def scene_setup(spec: SceneSpec, device="cpu") -> SceneSetup:
    """The seeded draws of `generate` up to rendering, in the same order (cheap: no rays)."""
    gen = torch.Generator().manual_seed(int(spec.seed) * 7919 + 17)
    N = spec.n_frames
    poses = _camera_path(spec, gen)
    path_xz = poses[:, [0, 2], 3]
    box_lo, box_hi, box_vel = _place_boxes(spec, path_xz, gen)
    n_obj = 2 + box_lo.shape[0]
    perm = make_permutation(gen, device)
    base = 0.25 + 0.5 * torch.rand(n_obj, 3, generator=gen, dtype=torch.float64)
    shift = 100.0 * torch.rand(n_obj, 3, 3, generator=gen, dtype=torch.float64)
    face_col = 0.1 + 0.8 * torch.rand(n_obj, 8, 3, generator=gen, dtype=torch.float64)
    moving = torch.zeros(n_obj, dtype=torch.bool)
    moving[2 + spec.n_static:] = True

    # pose perturbation (observed poses = true pose composed on the right)
    noisy = poses.clone()
    for i in range(N):
        w = torch.randn(3, generator=gen, dtype=torch.float64) * math.radians(spec.pose_rot_deg) / math.sqrt(3)
        t = torch.randn(3, generator=gen, dtype=torch.float64) * spec.pose_trans_m / math.sqrt(3)
        dT = torch.eye(4, dtype=torch.float64)
        dT[:3, :3] = _rodrigues(w)
        dT[:3, 3] = t
        noisy[i] = poses[i] @ dT
    noise_seed = int(torch.randint(0, 2**62, (1,), generator=gen))
    return SceneSetup(poses, noisy, box_lo, box_hi, box_vel, perm, base, shift, face_col, moving, noise_seed)


def true_depth(spec: SceneSpec, setup: SceneSetup, frame: int, pixels: torch.Tensor) -> torch.Tensor:
    """Noise-free z-depth of the given flat pixel indices (y W + x) of one frame (float64, CPU)."""
    W = spec.width
    fx = fy = spec.focal
    cx, cy = (W - 1) / 2.0, (spec.height - 1) / 2.0
    xs = (pixels % W).to(torch.float64)
    ys = (pixels // W).to(torch.float64)
    dirs = torch.stack([(xs - cx) / fx, (ys - cy) / fy, torch.ones_like(xs)], dim=-1)
    off = setup.box_vel * frame
    t, _, _ = _raycast(setup.poses[frame, :3, 3], setup.poses[frame, :3, :3], dirs, setup.box_lo + off,
                       setup.box_hi + off)
    return t


def generate(spec: SceneSpec, device="cpu", chunk_rays: int = 1 << 18) -> Clip:
    """Render a clip: clean radiance, z-depth, face ids; then add the noise models."""
    device = torch.device(device)
    W, H, N = spec.width, spec.height, spec.n_frames
    fx = fy = spec.focal
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0

    su = scene_setup(spec, device)
    poses, noisy, box_lo, box_hi, box_vel = su.poses, su.noisy, su.box_lo, su.box_hi, su.box_vel
    perm, base, shift, face_col, moving = su.perm, su.base, su.shift, su.face_col, su.moving
    noise_seed = su.noise_seed

    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(W, dtype=torch.float64), indexing="ij")
    dirs = torch.stack([(xs - cx) / fx, (ys - cy) / fy, torch.ones_like(xs)], dim=-1).reshape(-1, 3).to(device)
    base_d, shift_d, face_d = base.to(device), shift.to(device), face_col.to(device)
    moving_d = moving.to(device)

    clean = torch.empty(N, H * W, 3, dtype=torch.float32, device=device)
    depth_true = torch.empty(N, H * W, dtype=torch.float32, device=device)
    face_id = torch.empty(N, H * W, dtype=torch.int32, device=device)
    mov_mask = torch.empty(N, H * W, dtype=torch.bool, device=device)
    for n in range(N):
        o = poses[n, :3, 3].to(device)
        rot = poses[n, :3, :3].to(device)
        off = (box_vel * n).to(device)
        lo = box_lo.to(device) + off
        hi = box_hi.to(device) + off
        for s in range(0, H * W, chunk_rays):
            e = min(H * W, s + chunk_rays)
            t, obj, fc = _raycast(o, rot, dirs[s:e], lo, hi)
            pts = o[None, :] + t[:, None] * (dirs[s:e] @ rot.T)
            # moving objects are textured in their own (translating) frame
            boxi = torch.clamp(obj - 2, min=0)
            pobj = pts - torch.where((obj >= 2)[:, None], off[boxi], torch.zeros_like(pts))
            if spec.piecewise_constant:
                col = face_d[obj, fc]
            else:
                col = torch.empty(e - s, 3, dtype=torch.float64, device=device)
                for ch in range(3):
                    col[:, ch] = base_d[obj, ch] + 0.45 * fbm3(pobj + shift_d[obj, ch], perm, base_freq=0.5)
                col = col.clamp(0.05, 0.95)
            clean[n, s:e] = col.to(torch.float32)
            depth_true[n, s:e] = t.to(torch.float32)
            face_id[n, s:e] = (obj * 8 + fc).to(torch.int32)
            mov_mask[n, s:e] = moving_d[obj]

    # observation noise (drawn on the target device from a seeded generator)
    ngen = torch.Generator(device=device).manual_seed(noise_seed)
    clean64 = clean.to(torch.float64)
    clean_u8 = torch.round(clean64 * 255.0).clamp(0, 255).to(torch.uint8)
    rgb = torch.empty(N, H * W, 3, dtype=torch.uint8, device=device)
    dep = torch.empty(N, H * W, dtype=torch.float32, device=device)
    for n in range(N):
        g = torch.randn(H * W, 3, generator=ngen, dtype=torch.float64, device=device)
        rgb[n] = torch.round(255.0 * (clean64[n] + spec.colour_sigma * g)).clamp(0, 255).to(torch.uint8)
        gd = torch.randn(H * W, generator=ngen, dtype=torch.float64, device=device)
        dn = depth_true[n].to(torch.float64) * (1.0 + spec.depth_noise * gd)
        uo = torch.rand(H * W, generator=ngen, dtype=torch.float64, device=device)
        val = 2.0 + 18.0 * torch.rand(H * W, generator=ngen, dtype=torch.float64, device=device)
        dn = torch.where(uo < spec.outlier_frac, val, dn)
        dep[n] = dn.to(torch.float32)

    shp = (N, H, W)
    return Clip(
        spec=spec,
        rgb_u8=rgb.reshape(*shp, 3),
        depth=dep.reshape(shp),
        cam_to_world=noisy,
        fx=fx, fy=fy, cx=cx, cy=cy,
        clean_u8=clean_u8.reshape(*shp, 3),
        clean=clean.reshape(*shp, 3),
        depth_true=depth_true.reshape(shp),
        poses_true=poses,
        face_id=face_id.reshape(shp),
        moving_mask=mov_mask.reshape(shp),
        extra={"box_lo": box_lo, "box_hi": box_hi, "box_vel": box_vel},
    )
