"""Benchmark: scene-space gather + filter at 1920x1080 with a +-50 frame window.

One step = one output frame through the whole plain path: stage the frame that
enters the window (u8/f32 -> binary16), pose prep + count + scan, scatter, filter.
Inputs are synthetic (seeded ray-cast clip, 300 frames) and resident in HBM
before timing starts; the sample arena is sized by an untimed planning count.
The same frames also go through the fused gather + filter (no stored sets), the
last frame's sets through the paper's deblurring and inpainting filters, and,
unless --no-learned, the learned-weight filter.

Prints ONE JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _alg_bytes(n_pix: int, n_src: int, samples: int) -> dict:
    """Algorithmic (compulsory) HBM bytes per kernel for one output frame.

    count  : binary16 depth of every window frame (2 B/px) + int64 count per output pixel
    scatter: binary16 r,g,b,d of every window frame (8 B/px) + offsets (8 B/px)
             + records written (uint32 id + 4 x binary16 = 12 B/sample)
    filter : offsets (8 B/px) + records read (8 B/sample) + reference colour (8 B/px)
             + float32 RGB out (12 B/px)
    """
    return {
        "count": 2 * n_src * n_pix + 8 * n_pix,
        "scan": 16 * n_pix,
        "scatter": 8 * n_src * n_pix + 8 * n_pix + 12 * samples,
        "filter": 8 * n_pix + 8 * samples + 8 * n_pix + 12 * n_pix,
    }


GATHER_SOURCES = ("paper_2102_03011_amd/csrc/sg_kernels.hip", "paper_2102_03011_amd/csrc/sg_device.h",
                  "paper_2102_03011_amd/csrc/sg_internal.h", "include/scene_gather.h")


def gather_source_sha256() -> str:
    """Hash of every source the gather and filter kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    for rel in GATHER_SOURCES:
        h.update(rel.encode())
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def _measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size),
    or None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))["kernels"][kernel]
        sha = gather_source_sha256()
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha256") != sha:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def _host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _oracle_worker(args):
    """One process of the CPU baseline: the float64 oracle's gather and depth-weighted
    filter for a chunk of output pixels, reading the window planes from shared memory."""
    shm_name, shapes, f, prm, fx, fy, cx, cy, window, sigma_d, pixels = args
    import numpy as np
    from multiprocessing import shared_memory
    from oracle import filters as ofilters
    from oracle import gather as ogather
    shm = shared_memory.SharedMemory(name=shm_name)
    try:
        (cs, ds, ms) = shapes
        col = np.ndarray(cs, dtype=np.float64, buffer=shm.buf, offset=0)
        dep = np.ndarray(ds, dtype=np.float64, buffer=shm.buf, offset=col.nbytes)
        cams = np.ndarray(ms, dtype=np.float64, buffer=shm.buf, offset=col.nbytes + dep.nbytes)
        t0 = time.perf_counter()
        sets = ogather.gather_frame(col, dep, cams, fx, fy, cx, cy, f, ogather.GatherParams(**prm), pixels=pixels)
        out = ofilters.filter_sets(sets, col[f], window, sigma_d)
        dt = time.perf_counter() - t0
        seg = np.repeat(np.arange(sets.pixels.size), np.diff(sets.offsets))
        band = np.zeros(sets.pixels.size, bool)
        band[seg[sets.marginal]] = True
        band |= np.diff(sets.maybe_offsets) > 0
        certain = sets.ids[~sets.marginal]
        certain_off = np.concatenate([[0], np.cumsum(np.bincount(seg[~sets.marginal], minlength=sets.pixels.size))])
        return {"pixels": pixels, "offsets": sets.offsets, "ids": sets.ids, "certain_off": certain_off,
                "certain": certain, "maybe_off": sets.maybe_offsets, "maybe": sets.maybe_ids, "band": band,
                "out": out, "seconds": dt, "samples": int(sets.ids.size)}
    finally:
        shm.close()


def cpu_baseline(sg, clip, staged, wl, params, fparams, f: int, row_step: int, workers: int):
    """The float64 oracle on every `row_step`-th row of output frame f, one process
    per host core (spawned, reading the window planes from one shared-memory copy),
    and its comparison with the GPU's sets and filtered colours of the same pixels.
    Returns (cpu_baseline, oracle_error)."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor
    from multiprocessing import get_context, shared_memory
    from oracle import staging as ostaging

    # GPU side: the frame through the timed path's entry points, exact arena
    sets = sg.scene_gather(staged, f, f + 1, params)
    out = sg.scene_filter(staged, sets, fparams)
    torch.cuda.synchronize()
    sets.check()
    h, w = clip.height, clip.width
    g_off = sets.offsets.cpu().numpy()
    g_ids = sets.ids.cpu().numpy().view(np.uint32)
    g_out = out[0].reshape(-1, 3).cpu().numpy().astype(np.float64)
    del sets, out
    lo, hi = max(0, f - wl.window), min(clip.n_frames - 1, f + wl.window)
    n_win = hi - lo + 1
    cshape, dshape, mshape = (n_win, h, w, 3), (n_win, h, w), (n_win, 4, 4)
    nbytes = 8 * (int(np.prod(cshape)) + int(np.prod(dshape)) + int(np.prod(mshape)))
    shm = shared_memory.SharedMemory(create=True, size=nbytes)
    try:
        col = np.ndarray(cshape, dtype=np.float64, buffer=shm.buf, offset=0)
        dep = np.ndarray(dshape, dtype=np.float64, buffer=shm.buf, offset=col.nbytes)
        cams = np.ndarray(mshape, dtype=np.float64, buffer=shm.buf, offset=col.nbytes + dep.nbytes)
        for k in range(n_win):   # frame by frame: the staging conversion of the oracle
            col[k] = ostaging.colour_q(clip.rgb_u8[lo + k].cpu().numpy())
            dep[k] = ostaging.depth_q(clip.depth[lo + k].cpu().numpy())
        cams[:] = clip.cam_to_world[lo:hi + 1].cpu().numpy()
        rows = np.arange(0, h, row_step)
        pix = (rows[:, None] * w + np.arange(w)[None, :]).ravel()
        chunks = np.array_split(pix, 4 * workers)
        prm = {"window": wl.window, "radius": wl.radius, "tol": wl.tol, "z_near": wl.z_near}
        jobs = [(shm.name, (cshape, dshape, mshape), f - lo, prm, clip.fx, clip.fy, clip.cx, clip.cy, wl.window,
                 wl.sigma_d, c) for c in chunks]
        with ProcessPoolExecutor(max_workers=workers, mp_context=get_context("spawn")) as ex:
            list(ex.map(_oracle_worker, jobs[:workers]))         # start-up and imports, untimed
            t0 = time.perf_counter()
            parts = list(ex.map(_oracle_worker, jobs))
            dt = time.perf_counter() - t0
    finally:
        shm.close()
        shm.unlink()
    samples = sum(p["samples"] for p in parts)
    cpu_s = sum(p["seconds"] for p in parts)
    # oracle error of the GPU path on these pixels: membership (certain members
    # subset of the GPU's set subset of members + float32-band candidates) and colour
    bad_sets, checked, band_px, max_err, sum_err, n_err = 0, 0, 0, 0.0, 0.0, 0
    for p in parts:
        for k, q in enumerate(p["pixels"]):
            got = set(g_ids[g_off[q]:g_off[q + 1]].tolist())
            certain = set(p["certain"][p["certain_off"][k]:p["certain_off"][k + 1]].tolist())
            allowed = set(p["ids"][p["offsets"][k]:p["offsets"][k + 1]].tolist()) | \
                set(p["maybe"][p["maybe_off"][k]:p["maybe_off"][k + 1]].tolist())
            checked += 1
            if not (certain <= got <= allowed):
                bad_sets += 1
        e = np.abs(g_out[p["pixels"]] - p["out"]).max(axis=1)[~p["band"]]
        band_px += int(p["band"].sum())
        if e.size:
            max_err = max(max_err, float(e.max()))
            sum_err += float(e.sum())
            n_err += e.size
    base = {"value": samples / dt, "unit": "samples/s", "cores": workers, "kind": "oracle",
            "sample": f"frame {f}, every {row_step}th row ({pix.size} output pixels, {samples} samples), "
                      f"gather + depth-weighted filter, float64 numpy, {workers} processes, {dt:.1f} s wall, "
                      f"{cpu_s:.1f} s of process time",
            "seconds": dt, "host": _host_cpu_model(), "host_cores": os.cpu_count(),
            "samples_per_s_per_core": samples / cpu_s}
    err = {"frame": f, "pixels": int(pix.size), "sets_outside_bands_differing": bad_sets, "sets_checked": checked,
           "pixels_with_band_cases": band_px, "colour_max_abs_err": max_err,
           "colour_mean_abs_err": sum_err / max(n_err, 1), "colour_tolerance": 1e-3,
           "reference": "float64 oracle on the same binary16 planes (membership bands as the parity tests)"}
    return base, err


PAPER_REFERENCE = {
    "value": 3.4, "unit": "s per output frame", "application": "denoising", "hardware":
    "NVIDIA GeForce GTX 980 + Intel i7 3.2 GHz (Python with CUDA bindings)",
    "workload": "real 720p hand-held video, about 500 samples per set", "source": "Tab. time (Sec. 6)",
    "derived_samples_per_s": 1280 * 720 * 500 / 3.4,
    "note": "context only: other hardware, real video, paper's own parameters"}


MLP_FLOP_PER_SAMPLE = 2 * (8 * 64 + 64 * 64 + 64)   # 8 -> 64 -> 64 -> 1, multiply-adds x 2
BF16_DENSE_PEAK_TFLOPS = 2500.0


def fused_leg(sg, clip, staged, wl, params, fparams, timed, totals, stored_out, n_src) -> dict:
    """scene_gather_filter on the same output frames as the timed plain steps (the
    frame entering the window staged first, as there): whole step and kernel times,
    the fused kernel's roofline (it reads every source pixel of the window's blocks
    and writes the output: 8 B x sources x P + 8 B x P + 12 B x P), and its largest
    difference from the stored path's output on the last frame."""
    import torch
    n, h, w = clip.n_frames, clip.height, clip.width
    n_pix = h * w
    ws = sg.alloc_workspace(staged, 0, 1, params)
    out = torch.empty((1, h, w, 3), dtype=torch.float32, device=staged.rgbd.device)

    def step(f, ev=None):
        g = min(n - 1, f + wl.window)
        sg.scene_stage_into(staged, clip.rgb_u8[g], clip.depth[g], g)
        if ev is not None:
            ev[0].record()
        sg.scene_gather_filter(staged, f, f + 1, params, fparams, out=out, ws=ws)
        if ev is not None:
            ev[1].record()

    step(timed[0])
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in timed]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for k, f in enumerate(timed):
        step(f, evs[k])
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / len(timed)
    kms = sum(e[0].elapsed_time(e[1]) for e in evs) / len(timed)
    samples = sum(totals[f] for f in timed) / len(timed)
    alg = 8 * n_src * n_pix + 8 * n_pix + 12 * n_pix
    diff = (out.double() - stored_out.double()).abs().max().item()
    res = {"ms_per_step": ms, "kernel_ms": kms, "samples_per_s": samples / (ms / 1e3),
           "output_mpix_per_s": n_pix / (ms / 1e3) / 1e6,
           "roofline": {"bound": "hbm", "kernel": "gather_filter", "achieved": alg / (kms / 1e3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / (kms / 1e3) / 1e9 / HBM_PEAK_GBS,
                        "alg_bytes_per_launch": alg, "traffic": _measured_traffic("gather_filter")},
           "max_abs_diff_vs_stored_path": diff}
    log(f"fused gather + filter: {ms:.3f} ms/step (kernel {kms:.3f}), {res['output_mpix_per_s']:.0f} Mpix/s, "
        f"max |fused - stored| {diff:.2e}")
    return res


def filters_leg(sg, clip, staged, wl, arena, f, fparams, reps: int) -> dict:
    """The paper's other filters on the stored sets of output frame f (the last
    timed frame): the frame sharpness B(J) and a scene-space box mask over the
    whole clip, then `reps`
    calls each of the plain filter, the deblurring filter (Eq. 5: B(J) times the
    Eq. 4 weight with the paper's colour and frame sigmas) and inpainting (Eq. 8-9,
    two steps, sigma 55/255) under a moving box mask over ~10 % of each frame.
    HIP event times on the stream the kernels run on; algorithmic bytes of the
    frame filters: 12 B per record (colour + rho, id) + 28 B per pixel (offsets,
    own colour, output)."""
    import torch
    n, h, w = clip.n_frames, clip.height, clip.width
    dev = staged.rgbd.device
    sets = sg.SampleSets(f, f + 1, wl.window, arena.offsets, arena.ids, arena.crho, arena.status)
    n_rec = sets.total()
    out = torch.empty((1, h, w, 3), dtype=torch.float32, device=dev)
    mask = torch.zeros((n, h, w), dtype=torch.uint8, device=dev)
    bw, bh = w // 3, h // 3   # ~11 % of the frame, moving right 4 px per frame
    for j in range(n):
        xa = min(w, w // 6 + 4 * j)
        mask[j, h // 3:h // 3 + bh, xa:min(w, xa + bw)] = 1
    deblur = sg.FilterParams(sigma_d=fparams.sigma_d, sigma_c=200.0 / 255.0, sigma_t=20.0)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(k):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    bj = torch.empty((n,), dtype=torch.float32, device=dev)
    ms_sharp = timed(lambda: sg.scene_frame_sharpness(staged, out=bj), 3)
    box_mask = torch.empty_like(mask)
    ms_box = timed(lambda: sg.scene_box_mask(staged, (-1.0, -1.0, 0.5), (1.0, 1.0, 4.0), out=box_mask), 3)
    ms_plain = timed(lambda: sg.scene_filter(staged, sets, fparams, out=out), reps)
    ms_deblur = timed(lambda: sg.scene_filter_frames(staged, sets, deblur, bj, out=out), reps)
    ms_inpaint = timed(lambda: sg.scene_inpaint(staged, sets, mask, 55.0 / 255.0, 2, out=out), reps)
    ms_semi = timed(lambda: sg.scene_semi_transparent(staged, sets, mask, 80.0 / 255.0, 80.0 / 255.0, 2, out=out),
                    reps)
    # Eq. 4 with its scene-space term: the paper's sigma_xyz of 10 units of a scene scaled so
    # that 90 % of its points lie in a 10^3 cube is that cube's side in metres here
    side = scene_side_m(clip, staged)
    gp = sg.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near)
    ws = sg.alloc_workspace(staged, f, f + 1, gp)
    denoise7 = sg.FilterParams(sigma_d=math.inf, sigma_c=40.0 / 255.0, sigma_t=6.0)
    deblur7 = sg.FilterParams(sigma_d=math.inf, sigma_c=200.0 / 255.0, sigma_t=20.0)
    ms_xyz = timed(lambda: sg.scene_filter_xyz(staged, sets, gp, denoise7, side, ws=ws, out=out), reps)
    ms_xyz_deblur = timed(lambda: sg.scene_filter_xyz(staged, sets, gp, deblur7, side, frame_w=bj, ws=ws, out=out),
                          reps)
    alg = 12 * n_rec + 28 * h * w
    res = {"output_frame": f, "records": n_rec, "frames": n,
           "frame_sharpness_ms_per_clip": ms_sharp, "box_mask_ms_per_clip": ms_box,
           "plain_filter_ms": ms_plain, "deblur_filter_ms": ms_deblur,
           "deblur_roofline": {"bound": "hbm", "achieved": alg / (ms_deblur / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": alg / (ms_deblur / 1e3) / 1e9 / HBM_PEAK_GBS,
                               "alg_bytes_per_launch": alg},
           "inpaint_ms": ms_inpaint, "inpaint_masked_fraction": float(mask[f].float().mean().item()),
           "semi_transparent_ms": ms_semi, "scene_side_m": side,
           "eq4_scene_space_denoise_ms": ms_xyz, "eq5_scene_space_deblur_ms": ms_xyz_deblur}
    log(f"filters: B(J) {ms_sharp:.3f} ms/clip, box mask {ms_box:.3f} ms/clip, plain {ms_plain:.3f}, "
        f"deblur {ms_deblur:.3f}, "
        f"inpaint {ms_inpaint:.3f}, semi-transparent {ms_semi:.3f}, Eq. 4 with sigma_xyz {ms_xyz:.3f}, "
        f"Eq. 5 with sigma_xyz {ms_xyz_deblur:.3f} ms/frame")
    return res


def scene_side_m(clip, staged) -> float:
    """Side in metres of the cube that holds 90 % of the scene (the largest per-axis
    5 %-95 % range of the scene points of every 10th frame, from the stored depths)."""
    import torch
    h, w = clip.height, clip.width
    d = staged.rgbd_image()[::10, ..., 3].to(torch.float64)  # the depth channel
    ys, xs = torch.meshgrid(torch.arange(h, dtype=torch.float64, device=d.device),
                            torch.arange(w, dtype=torch.float64, device=d.device), indexing="ij")
    cams = staged.cam_to_world[::10].to(d.device)
    pts = []
    for k in range(d.shape[0]):
        dk = d[k]
        ok = torch.isfinite(dk) & (dk > 0)
        xc = torch.stack([dk * (xs - clip.cx) / clip.fx, dk * (ys - clip.cy) / clip.fy, dk], -1)[ok]
        pts.append(xc[::97] @ cams[k, :3, :3].T + cams[k, :3, 3])
    p = torch.cat(pts)
    return float(max(torch.quantile(p[:, k], 0.95) - torch.quantile(p[:, k], 0.05) for k in range(3)))


def frustum_leg(sg, clip, staged, f, window: int, reps: int) -> dict:
    """The depth-agnostic frustum gather (l = 3, depth range 0.01 .. 1000) of output
    frame f with a +-window window: count (carry, bucket, count, scan) and scatter,
    event-timed; records per pixel and gathered records per second."""
    import torch
    prm = sg.FrustumParams(window=window)
    ws = torch.empty(sg.scene_frustum_workspace_size(staged, f, prm), dtype=torch.uint8, device=staged.rgbd.device)
    sets = sg.scene_gather_frustum(staged, f, prm, ws=ws)
    torch.cuda.synchronize()
    sets.check()
    total = sets.total()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):   # count + scatter into the same arena, as the plain step reuses its own
        sg.scene_gather_frustum(staged, f, prm, ws=ws, sets=sets)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    sets.check()
    assert sets.total() == total
    n_pix = clip.height * clip.width
    res = {"window": window, "output_frame": f, "ms_per_frame": ms, "records": total,
           "records_per_pixel": total / n_pix, "records_per_s": total / (ms / 1e3),
           "workspace_gb": ws.numel() / 1e9}
    log(f"frustum gather +-{window}: {ms:.2f} ms/frame, {total / n_pix:.0f} records per pixel")
    return res


def depth_leg(sg, clip, staged, f, n_hyp: int, reps: int) -> dict:
    """Data-term depth of frame f over +-2 frames and n_hyp hypotheses spaced
    uniformly in inverse depth over [1, 30] m, event-timed."""
    import torch
    hyp = (1.0 / torch.linspace(1.0, 1.0 / 30.0, n_hyp, dtype=torch.float64)).to(torch.float32).cuda()
    sg.scene_estimate_depth(staged, f, 2, hyp)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        sg.scene_estimate_depth(staged, f, 2, hyp)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    n_pix = clip.height * clip.width
    res = {"window": 2, "hypotheses": n_hyp, "ms_per_frame": ms,
           "patch_costs_per_s": n_pix * n_hyp * 4 / (ms / 1e3)}
    log(f"depth estimate: {ms:.2f} ms/frame ({n_hyp} hypotheses, 4 frames)")
    return res


def learned_leg(sg, clip, staged, wl, params, fparams, timed, plain_ms, steps: int, with_curve: bool = True) -> dict:
    """The learned-weight filter on the same gathers (window +-w), timed like the plain
    step; PSNR of plain and learned on a few spread frames; and the learned path at
    the largest smaller window whose whole step is no slower than the plain step."""
    import torch
    from paper_2102_03011_amd import train

    try:
        mlp, meta = train.load_mlp()
    except OSError as e:
        return {"skipped": f"no trained weights ({e})"}
    dev = staged.rgbd.device
    n, h, w = clip.n_frames, clip.height, clip.width

    def arena_for(p, frames):
        plan = sg.alloc_sets(staged, 0, 1, p.window, 0)
        ws = sg.alloc_workspace(staged, 0, 1, p)
        tot = {}
        for f in frames:
            sg.scene_gather_count(staged, f, f + 1, p, plan, ws)
            tot[f] = plan.total()
        return sg.alloc_sets(staged, 0, 1, p.window, max(tot.values())), ws, tot

    def step_fn(p, arena, ws, out, learned: bool):
        def run(f, ev=None):
            sgs = sg.SampleSets(f, f + 1, p.window, arena.offsets, arena.ids, arena.crho, arena.status)
            g = min(n - 1, f + p.window)   # the frame entering the window, as in the plain step
            sg.scene_stage_into(staged, clip.rgb_u8[g], clip.depth[g], g)
            sg.scene_gather_count(staged, f, f + 1, p, sgs, ws)
            sg.scene_gather_scatter(staged, f, f + 1, p, sgs, ws)
            if ev is not None:
                ev[0].record()
            if learned:
                sg.scene_filter_learned(staged, sgs, p, mlp, ws=ws, out=out)
            else:
                sg.scene_filter(staged, sgs, fparams, out=out)
            if ev is not None:
                ev[1].record()
            return sgs
        return run

    def timed_run(run, frames):
        run(frames[0])
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in frames]
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for k, f in enumerate(frames):
            run(f, evs[k])
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / len(frames), sum(e[0].elapsed_time(e[1]) for e in evs) / len(frames)

    def psnr(x, ref):
        mse = torch.mean((x.to(torch.float64) - ref) ** 2).item()
        return 10 * math.log10(1 / mse)

    frames = timed[:steps]
    quality = sorted(set(timed[i * len(timed) // 4] for i in range(4)))
    out = torch.empty((1, h, w, 3), dtype=torch.float32, device=dev)
    arena, ws, tot = arena_for(params, sorted(set(frames) | set(quality)))
    ms_l, ms_lf = timed_run(step_fn(params, arena, ws, out, True), frames)
    samples = sum(tot[f] for f in frames) / len(frames)
    # quality on the same gathers
    ps_plain, ps_learned = [], []
    for f in quality:
        clean = clip.clean_u8[f].to(dev, torch.float64) / 255.0
        sgs = step_fn(params, arena, ws, out, False)(f)
        ps_plain.append(psnr(out[0], clean))
        sg.scene_filter_learned(staged, sgs, params, mlp, ws=ws, out=out)
        ps_learned.append(psnr(out[0], clean))
    res = {"weights": os.path.relpath(train.DEFAULT_WEIGHTS, ROOT), "trained_on": meta.get("clips"),
           "window": params.window, "ms_per_step": ms_l, "filter_ms": ms_lf,
           "samples_per_s": samples / (ms_l / 1e3),
           "mlp_tflops": samples * MLP_FLOP_PER_SAMPLE / (ms_lf / 1e3) / 1e12,
           "mlp_frac_of_bf16_peak": samples * MLP_FLOP_PER_SAMPLE / (ms_lf / 1e3) / 1e12 / BF16_DENSE_PEAK_TFLOPS,
           "quality_frames": quality, "psnr_plain_db": sum(ps_plain) / len(ps_plain),
           "psnr_learned_db": sum(ps_learned) / len(ps_learned)}
    log(f"learned w={params.window}: {ms_l:.2f} ms/step (filter {ms_lf:.2f}), PSNR plain "
        f"{res['psnr_plain_db']:.2f} learned {res['psnr_learned_db']:.2f}")
    del arena, ws
    # equal time: the largest window whose learned step fits the plain step's time;
    # the whole window / time / PSNR curve is reported
    curve = []
    for wq in (40, 30, 20, 12, 8, 6, 4, 3, 2, 1) if with_curve else ():
        if wq >= params.window:
            continue
        pq = sg.GatherParams(window=wq, radius=params.radius, tol=params.tol, z_near=params.z_near)
        arena, ws, totq = arena_for(pq, sorted(set(frames) | set(quality)))
        ms_q, ms_qf = timed_run(step_fn(pq, arena, ws, out, True), frames)
        pl = []
        for f in quality:
            clean = clip.clean_u8[f].to(dev, torch.float64) / 255.0
            step_fn(pq, arena, ws, out, True)(f)
            pl.append(psnr(out[0], clean))
        row = {"window": wq, "ms_per_step": ms_q, "filter_ms": ms_qf, "psnr_learned_db": sum(pl) / len(pl),
               "samples_per_pixel": sum(totq[f] for f in frames) / len(frames) / (h * w)}
        curve.append(row)
        log(f"learned w={wq}: {ms_q:.2f} ms/step, PSNR {row['psnr_learned_db']:.2f} "
            f"(plain w={params.window}: {plain_ms:.2f} ms, {res['psnr_plain_db']:.2f} dB)")
        if ms_q <= plain_ms and "equal_time" not in res:
            res["equal_time"] = {**row, "plain_ms_per_step": plain_ms,
                                 "psnr_plain_db_full_window": res["psnr_plain_db"]}
        del arena, ws
    res["curve"] = curve
    return res


def batched_main(args) -> int:
    """The 32 uneven clips (640x360 .. 1920x1080, 30-150 frames, windows 10-40) as
    one batch: one step = one output frame of every clip through pose prep, count,
    scan, scatter and filter, replayed from a captured graph with new frames each
    step. The same work through the single-clip entry points, clip after clip, is
    timed beside it."""
    import torch
    import paper_2102_03011_amd as sg
    from scenegen import configs, generate

    dev = torch.device("cuda:0")
    wls = configs.batched_clips()
    t0 = time.perf_counter()
    staged, lengths = [], []
    for wl in wls:
        clip = generate(wl.spec, device=dev, chunk_rays=1 << 20)
        staged.append(sg.scene_stage(clip.rgb_u8, clip.depth, clip.cam_to_world.to(dev), clip.fx, clip.fy,
                                     clip.cx, clip.cy))
        lengths.append(clip.n_frames)
        del clip
    torch.cuda.synchronize()
    log(f"generated {len(wls)} clips in {time.perf_counter() - t0:.1f} s")
    params = [sg.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near) for wl in wls]
    fparams = [sg.FilterParams(sigma_d=wl.sigma_d) for wl in wls]
    b = sg.Batch(staged, params, fparams, 1)
    n_steps = args.warmup + args.steps
    frames = [[(n // 2 + k - n_steps // 2) % n for n in lengths] for k in range(n_steps)]
    plan = b.alloc_io(1, with_out=False)
    totals = []
    for f0 in frames:
        b.set_frames(f0)
        totals.append(b.count(plan))
    del plan
    io = b.alloc_io(max(totals))
    b.set_frames(frames[0])
    cfg = b.autotune(io)
    passes = b.time_passes(io)
    log(f"autotuned config {cfg}; passes (ms) {passes}")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.capture(io)
        for k in range(args.warmup):
            b.set_frames(frames[k])
            b.gather(io)
        stream.synchronize()
        io.check()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for k in range(args.warmup, n_steps):
            b.set_frames(frames[k])
            b.gather(io)
        stop.record(stream)
        stream.synchronize()
    io.check()
    ms_step = start.elapsed_time(stop) / args.steps
    samples = sum(totals[args.warmup:]) / args.steps
    # the same steps through the single-clip entry points, clip after clip
    arenas = []
    for c, wl in enumerate(wls):
        cap = 0
        plan = sg.alloc_sets(staged[c], 0, 1, wl.window, 0)
        ws = sg.alloc_workspace(staged[c], 0, 1, params[c])
        for f0 in frames[args.warmup:]:
            sg.scene_gather_count(staged[c], f0[c], f0[c] + 1, params[c], plan, ws)
            cap = max(cap, plan.total())
        arenas.append((sg.alloc_sets(staged[c], 0, 1, wl.window, cap), ws,
                       torch.empty((1, wl.spec.height, wl.spec.width, 3), dtype=torch.float32, device=dev)))
    del io

    def solo_step(f0):
        for c in range(len(wls)):
            a, ws, out = arenas[c]
            sets = sg.SampleSets(f0[c], f0[c] + 1, params[c].window, a.offsets, a.ids, a.crho, a.status)
            sg.scene_gather_count(staged[c], f0[c], f0[c] + 1, params[c], sets, ws)
            sg.scene_gather_scatter(staged[c], f0[c], f0[c] + 1, params[c], sets, ws)
            sg.scene_filter(staged[c], sets, fparams[c], out=out)

    solo_step(frames[0])
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for k in range(args.warmup, n_steps):
        solo_step(frames[k])
    stop.record()
    torch.cuda.synchronize()
    solo_ms = start.elapsed_time(stop) / args.steps
    # per-pass split of the single-clip path (one more step, events between passes)
    solo_passes = {"count": 0.0, "scatter": 0.0, "filter": 0.0}
    evs = []
    for c in range(len(wls)):
        a, ws, out = arenas[c]
        fc = frames[args.warmup][c]
        sets = sg.SampleSets(fc, fc + 1, params[c].window, a.offsets, a.ids, a.crho, a.status)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        sg.scene_gather_count(staged[c], fc, fc + 1, params[c], sets, ws)
        e[1].record()
        sg.scene_gather_scatter(staged[c], fc, fc + 1, params[c], sets, ws)
        e[2].record()
        sg.scene_filter(staged[c], sets, fparams[c], out=out)
        e[3].record()
        evs.append(e)
    torch.cuda.synchronize()
    for e in evs:
        solo_passes["count"] += e[0].elapsed_time(e[1])   # count includes the scan
        solo_passes["scatter"] += e[1].elapsed_time(e[2])
        solo_passes["filter"] += e[2].elapsed_time(e[3])
    pix = b.total_pixels
    res = {
        "metric": "gathered samples/s (32 uneven clips per step, one persistent launch per pass, graph replay)",
        "value": samples / (ms_step / 1e3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (binary16 storage)",
        "data": "synthetic (seeded ray-cast clips; no real video)",
        "config": {"workload": "batched uneven clips", "clips": len(wls), "output_pixels_per_step": pix,
                   "resolutions": sorted({f"{wl.spec.width}x{wl.spec.height}" for wl in wls}),
                   "frames": [min(lengths), max(lengths)], "windows": [min(p.window for p in params),
                                                                       max(p.window for p in params)],
                   "autotuned": {"count_tile_waves": cfg[0], "count_frame_unroll": cfg[1],
                                 "scatter_tile_waves": cfg[2]}},
        "output_mpix_per_s": pix / (ms_step / 1e3) / 1e6,
        "samples_per_step": samples,
        "pass_ms_eager": passes,
        "solo_ms_per_step": solo_ms,
        "solo_pass_ms": solo_passes,
        "speedup_vs_solo": solo_ms / ms_step,
        "gpu": torch.cuda.get_device_name(0),
    }
    b.close()
    print(json.dumps(res), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=300, help="clip length (the workload uses 300)")
    ap.add_argument("--chunk-rays", type=int, default=1 << 20,
                    help="rays per generation launch (larger = fewer launches, e.g. under a counter profiler)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-row-step", type=int, default=4,
                    help="the CPU baseline runs the oracle on every n-th row of one output frame")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes (0: one per host core available, at most 16)")
    ap.add_argument("--workload", choices=("full", "batched"), default="full",
                    help="full: the 1080p +-50 headline workload; batched: 32 uneven clips per step")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-weight filter leg")
    ap.add_argument("--learned-steps", type=int, default=5)
    ap.add_argument("--no-fused", action="store_true", help="skip the fused gather + filter leg")
    ap.add_argument("--depth-hypotheses", type=int, default=32,
                    help="also time the data-term depth estimate with this many hypotheses (0: skip)")
    ap.add_argument("--frustum-window", type=int, default=10,
                    help="also time the depth-agnostic frustum gather with this window (0: skip)")
    ap.add_argument("--no-filters", action="store_true",
                    help="skip the deblurring / inpainting filters leg")
    ap.add_argument("--no-curve", action="store_true",
                    help="learned leg at the workload's window only (no smaller-window curve)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, run one plain 1 GiB elementwise copy and one gather of 2^24 random "
                         "64-byte rows (counter calibration for streaming and scattered reads)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(output frames would shard across GPUs without any exchange)", file=sys.stderr)
        return 2

    if args.workload == "batched":
        return batched_main(args)

    import torch
    import paper_2102_03011_amd as sg
    from scenegen import configs, generate

    dev = torch.device("cuda:0")
    wl = configs.full_scale(n_frames=args.frames)
    t0 = time.perf_counter()
    clip = generate(wl.spec, device=dev, chunk_rays=args.chunk_rays)
    torch.cuda.synchronize()
    log(f"generated {wl.name} in {time.perf_counter() - t0:.1f} s")
    n, h, w = clip.n_frames, clip.height, clip.width
    n_pix = h * w
    c2w = clip.cam_to_world.to(dev)
    staged = sg.scene_stage(clip.rgb_u8, clip.depth, c2w, clip.fx, clip.fy, clip.cx, clip.cy)
    params = sg.GatherParams(window=wl.window, radius=wl.radius, tol=wl.tol, z_near=wl.z_near)
    fparams = sg.FilterParams(sigma_d=wl.sigma_d)

    first = wl.window
    span = max(1, n - 2 * wl.window)
    frames = [first + (k % span) for k in range(args.warmup + args.steps)]
    ws = sg.alloc_workspace(staged, 0, 1, params)
    # planning pass (untimed): exact totals per output frame size the arena
    plan = sg.alloc_sets(staged, 0, 1, wl.window, 0)
    totals = {}
    for f in sorted(set(frames)):
        sg.scene_gather_count(staged, f, f + 1, params, plan, ws)
        totals[f] = plan.total()
    cap = max(totals.values())
    arena = sg.alloc_sets(staged, 0, 1, wl.window, cap)
    out = torch.empty((1, h, w, 3), dtype=torch.float32, device=dev)
    log(f"samples/frame min {min(totals.values())} max {cap} ({cap / n_pix:.1f} per pixel)")

    def run_step(f, ev=None):
        # stage the frame entering the window (streaming order); same bytes as before
        g = min(n - 1, f + wl.window)
        sgs = sg.SampleSets(f, f + 1, wl.window, arena.offsets, arena.ids, arena.crho, arena.status)
        if ev is not None:
            ev[0].record()
        sg.scene_stage_into(staged, clip.rgb_u8[g], clip.depth[g], g)
        if ev is not None:
            ev[1].record()
        sg.scene_gather_count(staged, f, f + 1, params, sgs, ws)
        if ev is not None:
            ev[2].record()
        sg.scene_gather_scatter(staged, f, f + 1, params, sgs, ws)
        if ev is not None:
            ev[3].record()
        sg.scene_filter(staged, sgs, fparams, out=out)
        if ev is not None:
            ev[4].record()

    for k in range(args.warmup):
        run_step(frames[k])
    torch.cuda.synchronize()
    arena.check()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    timed = frames[args.warmup:]
    torch.cuda.synchronize()
    start.record()
    for k, f in enumerate(timed):
        run_step(f, evs[k])
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    arena.check()
    parts = {"stage": 0.0, "count": 0.0, "scatter": 0.0, "filter": 0.0}
    for ev in evs:
        parts["stage"] += ev[0].elapsed_time(ev[1])
        parts["count"] += ev[1].elapsed_time(ev[2])
        parts["scatter"] += ev[2].elapsed_time(ev[3])
        parts["filter"] += ev[3].elapsed_time(ev[4])
    per = {k: v / args.steps for k, v in parts.items()}
    samples = sum(totals[f] for f in timed)
    ms_step = total_ms / args.steps
    value = samples / (total_ms / 1e3)
    mpix = n_pix * args.steps / (total_ms / 1e3) / 1e6

    # PSNR of the last filtered frame vs the clean radiance (quantised like the input)
    f_last = timed[-1]
    clean = clip.clean_u8[f_last].to(torch.float64) / 255.0
    noisy = staged.rgbd_image()[f_last, ..., :3].to(torch.float64)
    mse_f = torch.mean((out[0].to(torch.float64) - clean) ** 2).item()
    mse_n = torch.mean((noisy - clean) ** 2).item()

    n_src = min(n - 1, f_last + wl.window) - max(0, f_last - wl.window) + 1
    mean_s = samples / args.steps
    alg = _alg_bytes(n_pix, n_src, int(mean_s))
    dom = max(("count", "scatter", "filter"), key=lambda k: per[k])
    achieved = alg[dom] / (per[dom] / 1e3) / 1e9
    path_bytes = alg["count"] + alg["scan"] + alg["scatter"] + alg["filter"] + 18 * n_pix
    res = {
        "metric": "gathered samples/s (1080p, +-50-frame window, plain depth-weighted filter)",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (binary16 storage)",
        "data": "synthetic (seeded ray-cast clip, Perlin-textured boxes; no real video)",
        "config": {"workload": wl.name, "width": w, "height": h, "frames": n, "window": wl.window,
                   "radius": wl.radius, "tol": wl.tol, "sigma_d": wl.sigma_d,
                   "static_boxes": wl.spec.n_static, "moving_boxes": wl.spec.n_moving,
                   "colour_sigma_255": round(wl.spec.colour_sigma * 255, 3),
                   "depth_noise": wl.spec.depth_noise, "outliers": wl.spec.outlier_frac},
        "output_mpix_per_s": mpix,
        "samples_per_pixel": mean_s / n_pix,
        "per_kernel_ms": per,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": _measured_traffic(dom),
                     "alg_bytes_per_launch": alg[dom]},
        "path_hbm_frac": path_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "psnr_db": {"noisy_input": 10 * math.log10(1 / mse_n), "plain_filter": 10 * math.log10(1 / mse_f)},
        "gpu": torch.cuda.get_device_name(0),
    }
    if args.depth_hypotheses > 0:
        res["depth"] = depth_leg(sg, clip, staged, timed[-1], args.depth_hypotheses, max(2, args.steps // 2))
    if args.frustum_window > 0:
        res["frustum"] = frustum_leg(sg, clip, staged, timed[-1], args.frustum_window, max(2, args.steps // 2))
    if not args.no_filters:
        res["filters"] = filters_leg(sg, clip, staged, wl, arena, timed[-1], fparams, max(3, args.steps))
    if not args.no_fused:
        res["fused"] = fused_leg(sg, clip, staged, wl, params, fparams, timed, totals, out, n_src)
    if not args.no_learned:
        res["learned"] = learned_leg(sg, clip, staged, wl, params, fparams, frames[args.warmup:], ms_step,
                                     args.learned_steps, with_curve=not args.no_curve)
    if "fused" in res and "learned" in res and "curve" in res["learned"]:
        # the learned path against the fused plain path's time as well: the largest
        # window whose learned step is no slower (None if none is)
        fit = [r for r in res["learned"]["curve"] if r["ms_per_step"] <= res["fused"]["ms_per_step"]]
        res["learned"]["equal_time_vs_fused_plain"] = (
            {**max(fit, key=lambda r: r["window"]), "fused_plain_ms_per_step": res["fused"]["ms_per_step"]}
            if fit else None)
    if args.copy_probe:
        x = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        # scattered reads: 2^24 rows of 64 B (1 GiB) read in a random order, written in order
        rows = x.view(1 << 24, 16)
        idx = torch.randperm(1 << 24, device=dev, generator=torch.Generator(device=dev).manual_seed(3))
        torch.cuda.synchronize()
        torch.index_select(rows, 0, idx, out=y.view(1 << 24, 16))
        torch.cuda.synchronize()
        del x, y, rows, idx
    res["paper_reference"] = PAPER_REFERENCE
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(16, len(os.sched_getaffinity(0)))
        log(f"timing the float64 oracle on a bounded sample ({workers} processes) and comparing it with the GPU")
        res["cpu_baseline"], res["oracle_error"] = cpu_baseline(sg, clip, staged, wl, params, fparams, timed[0],
                                                                args.cpu_row_step, workers)
        log(f"oracle: {res['cpu_baseline']['value']:.3g} samples/s on {workers} processes; "
            f"error {res['oracle_error']}")
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
