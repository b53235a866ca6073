"""Training of the per-sample weighting MLP on sample sets that the gather itself
produces from synthetic clips with known clean radiance.

    python -m paper_2102_03011_amd.train [--clips 200] [--out FILE]

Every arithmetic step runs in the library's kernels: the gather (count / scan /
scatter), the feature statistics (scene_feature_moments), the forward/backward
and Adam step (scene_mlp_train_step) and, for evaluation, the plain and learned
filters. Python only draws clips, frames and pixel batches and moves tensors.

Training data: 640x360 clips of 60 frames (seeds 1000 + i), window +-30, 3x3
source block, tolerance 1% of depth; evaluation: held-out clips (seeds 2000 + i),
PSNR of the plain depth-weighted filter and of the learned filter against the
clean radiance.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import time

import numpy as np
import torch

import paper_2102_03011_amd as sg
from scenegen import configs, generate

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "mlp_640x360_mix.npz")
FORMAT_VERSION = 1


# ---------------------------------------------------------------------------
# checkpoint

def save_mlp(path: str, params: sg.MLPParams, meta: dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, w_bf16=params.w.cpu().numpy().view(np.uint16), b=params.b.cpu().numpy(),
             meta=np.frombuffer(json.dumps({"format": FORMAT_VERSION, **meta}).encode(), dtype=np.uint8))


def load_mlp(path: str = DEFAULT_WEIGHTS, device="cuda") -> tuple[sg.MLPParams, dict]:
    """Weights saved by save_mlp (plain arrays; nothing is unpickled)."""
    z = np.load(path, allow_pickle=False)
    meta = json.loads(bytes(z["meta"]).decode())
    if meta.get("format") != FORMAT_VERSION:
        raise ValueError(f"{path}: unsupported weight format {meta.get('format')}")
    w = torch.from_numpy(z["w_bf16"].astype(np.uint16).view(np.int16).copy()).to(device)
    b = torch.from_numpy(z["b"].astype(np.float32)).to(device)
    if w.numel() != sg.SG_MLP_NW or b.numel() != sg.SG_MLP_NB:
        raise ValueError(f"{path}: wrong parameter counts")
    return sg.MLPParams(w.contiguous(), b.contiguous()), meta


def init_params(moments: torch.Tensor, seed: int, device="cuda") -> sg.MLPParams:
    """He initialisation (normal, fan-in), zero biases; the input standardisation
    from the feature moments (computed by the library on the device)."""
    g = np.random.default_rng(seed)
    w1 = g.normal(size=(8, 64)) * math.sqrt(2.0 / 8)
    w2 = g.normal(size=(64, 64)) * math.sqrt(2.0 / 64)
    w3 = g.normal(size=64) * math.sqrt(1.0 / 64)
    z = np.zeros(64)
    p = sg.MLPParams.from_arrays(w1, z, w2, z, w3, 0.0, np.zeros(8), np.ones(8), device=device)
    sg.scene_mlp_standardise(moments, p)
    return p


# ---------------------------------------------------------------------------
# data

class FrameSets:
    """One clip staged on the device and the gathered sets of one output frame."""

    def __init__(self, clip, staged, wl, f, window=None):
        self.clip, self.staged, self.f = clip, staged, f
        w = wl.window if window is None else window
        self.params = sg.GatherParams(window=w, radius=wl.radius, tol=wl.tol, z_near=wl.z_near)
        self.ws = sg.alloc_workspace(staged, f, f + 1, self.params)
        self.sets = sg.scene_gather(staged, f, f + 1, self.params, ws=self.ws)
        self.sets.check()
        self.n = clip.height * clip.width
        self.clean = clip.clean[f].reshape(-1, 3).to(staged.rgbd.device, torch.float32)
        counts = self.sets.offsets[1:] - self.sets.offsets[:-1]
        self.nonempty = torch.nonzero(counts > 0).flatten().to(torch.int32)


def training_workload(i: int, noise_mix: bool):
    """Training clip i; with noise_mix its noise levels and moving objects are drawn
    per clip (colour sigma 4-12/255, depth noise 1-4 %, outliers 0.5-2 %, 0-3 movers)."""
    wl = configs.learned_train(i)
    if noise_mix:
        g = np.random.default_rng(50_000 + i)
        wl.spec = dataclasses.replace(wl.spec, colour_sigma=g.uniform(4, 12) / 255.0,
                                      depth_noise=g.uniform(0.01, 0.04), outlier_frac=g.uniform(0.005, 0.02),
                                      n_moving=int(g.integers(0, 4)))
    return wl


def make_clip(wl, device="cuda"):
    clip = generate(wl.spec, device=device, chunk_rays=1 << 20)
    staged = sg.scene_stage(clip.rgb_u8, clip.depth, clip.cam_to_world.to(device), clip.fx, clip.fy,
                            clip.cx, clip.cy)
    return clip, staged


def sample_pixels(fs: FrameSets, n: int, gen: torch.Generator) -> torch.Tensor:
    k = torch.randint(0, fs.nonempty.numel(), (n,), generator=gen, device="cpu").to(fs.nonempty.device)
    return fs.nonempty[k].contiguous()


# ---------------------------------------------------------------------------

def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    mse = torch.mean((a.double() - b.double()) ** 2).item()
    return 10.0 * math.log10(1.0 / mse) if mse > 0 else math.inf


def evaluate(params: sg.MLPParams, n_clips: int = 20, frames_per_clip: int = 3, seed: int = 7, log=print,
             windows=(30,)):
    """PSNR (input, plain filter, learned filter) on held-out clips, per window."""
    rng = np.random.default_rng(seed)
    rows = {w: [] for w in windows}
    for i in range(n_clips):
        wl = configs.learned_train(i, held_out=True)
        clip, staged = make_clip(wl)
        for f in sorted(rng.choice(clip.n_frames, size=frames_per_clip, replace=False).tolist()):
            clean = clip.clean[f].to(staged.rgbd.device)
            noisy = clip.rgb_u8[f].to(staged.rgbd.device).double() / 255.0
            for w in windows:
                fs = FrameSets(clip, staged, wl, f, window=w)
                plain = sg.scene_filter(staged, fs.sets, sg.FilterParams(sigma_d=wl.sigma_d))[0]
                learned = sg.scene_filter_learned(staged, fs.sets, fs.params, params, ws=fs.ws)[0]
                rows[w].append((psnr(noisy, clean), psnr(plain, clean), psnr(learned, clean)))
        del clip, staged
        log(f"eval: held-out clip {i + 1} of {n_clips} done")
    out = {"clips": n_clips, "frames": n_clips * frames_per_clip}
    for w in windows:
        r = np.array(rows[w])
        out[f"w{w}"] = {"psnr_input": float(r[:, 0].mean()), "psnr_plain": float(r[:, 1].mean()),
                        "psnr_learned": float(r[:, 2].mean()),
                        "learned_minus_plain_min": float((r[:, 2] - r[:, 1]).min()),
                        "learned_beats_plain_frames": int((r[:, 2] > r[:, 1]).sum())}
    log(f"eval: {json.dumps(out)}")
    return out


def train(n_clips: int = 200, frames_per_clip: int = 4, steps_per_frame: int = 8, batch: int = 4096,
          lr: float = 2e-3, lr_final: float = 2e-4, stats_clips: int = 8, seed: int = 0, log=print,
          windows=(30,), noise_mix: bool = False):
    t0 = time.time()
    gen = torch.Generator().manual_seed(seed)
    rng = np.random.default_rng(seed)
    # feature statistics over a few clips
    moments = None
    for i in range(stats_clips):
        wl = training_workload(i, noise_mix)
        clip, staged = make_clip(wl)
        for f in rng.choice(clip.n_frames, size=2, replace=False).tolist():
            fs = FrameSets(clip, staged, wl, f, window=int(rng.choice(windows)))
            moments = sg.scene_feature_moments(staged, fs.sets, fs.params, sample_pixels(fs, batch, gen),
                                               moments=moments, ws=fs.ws)
    init = init_params(moments, seed)
    std_b = init.b.detach().cpu().numpy()
    log(f"feature mean {np.array2string(std_b[132:140], precision=4)} "
        f"1/std {np.array2string(std_b[140:148], precision=4)}")
    state = sg.MLPTrainState(init)
    total = n_clips * frames_per_clip * steps_per_frame
    losses = []
    step = 0
    for i in range(n_clips):
        wl = training_workload(i, noise_mix)
        clip, staged = make_clip(wl)
        for f in rng.choice(clip.n_frames, size=frames_per_clip, replace=False).tolist():
            fs = FrameSets(clip, staged, wl, f, window=int(rng.choice(windows)))
            for _ in range(steps_per_frame):
                cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / max(total - 1, 1)))
                idx = sample_pixels(fs, batch, gen)
                sg.scene_mlp_train_step(staged, fs.sets, fs.params, idx, fs.clean[idx.long()].contiguous(),
                                        state, cur, ws=fs.ws)
                step += 1
            losses.append(float(state.loss.item()))
        del clip, staged
        if (i + 1) % 10 == 0 or i + 1 == n_clips:
            log(f"clip {i + 1}/{n_clips}  step {step}  loss {np.mean(losses[-10 * frames_per_clip:]):.3e}  "
                f"{time.time() - t0:.0f}s")
    meta = {"clips": n_clips, "frames_per_clip": frames_per_clip, "steps": step, "batch": batch, "lr": lr,
            "lr_final": lr_final, "seed": seed, "windows": list(windows), "noise_mix": noise_mix,
            "mean": std_b[132:140].tolist(), "inv_std": std_b[140:148].tolist(),
            "final_loss": float(np.mean(losses[-20:])), "seconds": time.time() - t0}
    return state.params, meta


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--clips", type=int, default=200)
    ap.add_argument("--frames-per-clip", type=int, default=4)
    ap.add_argument("--steps-per-frame", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-clips", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--windows", default="30", help="comma-separated windows drawn per training frame")
    ap.add_argument("--noise-mix", action="store_true", help="draw noise levels and movers per clip")
    ap.add_argument("--eval-windows", default="30")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval-only", metavar="WEIGHTS", default=None,
                    help="no training: evaluate these weights on --eval-clips held-out clips and print the result")
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("training needs a GPU")
    if a.eval_only is not None:
        params, _ = load_mlp(a.eval_only)
        res = evaluate(params, a.eval_clips, log=lambda s: print(s, flush=True),
                       windows=tuple(int(x) for x in a.eval_windows.split(",")))
        print(json.dumps({"weights": a.eval_only, "eval": res}), flush=True)
        return
    windows = tuple(int(x) for x in a.windows.split(","))
    params, meta = train(a.clips, a.frames_per_clip, a.steps_per_frame, a.batch, a.lr, a.lr / 10, seed=a.seed,
                         log=lambda s: print(s, flush=True), windows=windows, noise_mix=a.noise_mix)
    if a.eval_clips > 0:
        meta["eval"] = evaluate(params, a.eval_clips, log=lambda s: print(s, flush=True),
                                windows=tuple(int(x) for x in a.eval_windows.split(",")))
    save_mlp(a.out, params, meta)
    print(json.dumps({k: v for k, v in meta.items() if k not in ("mean", "std")}), flush=True)


if __name__ == "__main__":
    main()
