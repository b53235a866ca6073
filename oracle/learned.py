"""Learned per-sample weights for the sample-set filter (test infrastructure only).

The paper's filter is a weighted mean of a sample set (Sec. 5, Eq. 3) with a
hand-set weight (Sec. 5, Eq. 4). Here the weight comes from a small MLP on
eight per-sample features, normalised over the set with a softmax:

  O(p) = sum_s a_s c_s,  a = softmax_s(m_s),  m_s = MLP(standardise(x_s)),
  MLP: 8 -> 64 -> 64 -> 1, GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2.

Features of sample s (source frame J, source pixel q) of output pixel p in frame f:
  x1 = rho_s, the relative depth residual D^J(q) / z - 1
  x2 = |c_s - med(S)|_2, med the per-channel lower median (sorted[(n - 1) // 2])
  x3 = |J - f| / w
  x4 = |q - (u, v)|_2, distance from q to the unrounded projection in J (pixels)
  x5 = 1 - cos of the angle at X between the rays from the camera centres of f and J
  x6 = |grad D^J|(q) / D^J(q), central differences (one-sided where a neighbour is
       outside the image or has no valid depth; 0 when both are missing)
  x7 = log(1 + n) / log(1 + (2r + 1)^2 (2w + 1)),  n = |S|
  x8 = (J - f) / w
(w = 0 gives x3 = x8 = 0.) Readings of the feature list (the workload names the
features only): lower median, L2 colour distance, signed vs absolute frame term,
and the view-angle term as 1 - cos (an affine image of the cosine, which the
standardisation absorbs; near 1 the cosine itself is ill-conditioned in float32).

Precision: the weights are values representable in bfloat16 (the caller rounds
them; bf16_round below); features and activations are exact float64 here. The
kernels carry features and layer-1 activations as bfloat16 hi/lo pairs (about 16
significant bits), so they evaluate this same function to float32-level error.
Training minimises L = sum_p |O(p) - G(p)|^2 / (3 P) (P pixels of the
minibatch; an empty set contributes nothing) with Adam
(beta1 0.9, beta2 0.999, eps 1e-8) on float32 master weights.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import erf as _erf

from . import gather as _gather
from . import poses as _poses

N_FEAT, N_HID = 8, 64
_SQRT2 = math.sqrt(2.0)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / _SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / _SQRT2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


@dataclass
class MLP:
    w1: np.ndarray      # [8, 64]
    b1: np.ndarray      # [64]
    w2: np.ndarray      # [64, 64]
    b2: np.ndarray      # [64]
    w3: np.ndarray      # [64]
    b3: float
    mean: np.ndarray    # [8] feature mean
    std: np.ndarray     # [8] feature standard deviation

    def copy(self):
        return MLP(self.w1.copy(), self.b1.copy(), self.w2.copy(), self.b2.copy(), self.w3.copy(),
                   float(self.b3), self.mean.copy(), self.std.copy())


def init_mlp(seed: int, mean=None, std=None) -> MLP:
    rng = np.random.default_rng(seed)
    w1 = rng.normal(size=(N_FEAT, N_HID)) * math.sqrt(2.0 / N_FEAT)
    w2 = rng.normal(size=(N_HID, N_HID)) * math.sqrt(2.0 / N_HID)
    w3 = rng.normal(size=N_HID) * math.sqrt(1.0 / N_HID)
    z = np.zeros(N_HID)
    return MLP(w1, z.copy(), w2, z.copy(), w3, 0.0,
               np.zeros(N_FEAT) if mean is None else np.asarray(mean, float),
               np.ones(N_FEAT) if std is None else np.asarray(std, float))


# ---------------------------------------------------------------------------
# features

def lower_median(colour: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Per-set, per-channel lower median: sorted values[(n - 1) // 2]; [n_sets, 3]."""
    n = offsets.size - 1
    out = np.zeros((n, 3))
    for i in range(n):
        s, e = offsets[i], offsets[i + 1]
        if e > s:
            srt = np.sort(colour[s:e], axis=0)
            out[i] = srt[(e - s - 1) // 2]
    return out


def _depth_gradient(dplane: np.ndarray, qx: np.ndarray, qy: np.ndarray) -> np.ndarray:
    h, w = dplane.shape

    def val(x, y):
        ok = (x >= 0) & (x < w) & (y >= 0) & (y < h)
        v = np.full(x.shape, np.nan)
        v[ok] = dplane[y[ok], x[ok]]
        good = ok & np.isfinite(v) & (v > 0)
        return np.where(good, v, np.nan), good

    d0, _ = val(qx, qy)

    def axis_grad(dx, dy):
        dp, gp = val(qx + dx, qy + dy)
        dm, gm = val(qx - dx, qy - dy)
        g = np.zeros(qx.shape)
        both = gp & gm
        g[both] = 0.5 * (dp[both] - dm[both])
        only_p = gp & ~gm
        g[only_p] = dp[only_p] - d0[only_p]
        only_m = gm & ~gp
        g[only_m] = d0[only_m] - dm[only_m]
        return g

    gx = axis_grad(1, 0)
    gy = axis_grad(0, 1)
    return np.sqrt(gx * gx + gy * gy) / d0


def features(pix_of: np.ndarray, ids: np.ndarray, rho: np.ndarray, colour: np.ndarray,
             offsets: np.ndarray, pixels: np.ndarray, f: int, depth: np.ndarray,
             cam_to_world: np.ndarray, fx, fy, cx, cy, window: int, radius: int) -> np.ndarray:
    """Raw (unstandardised) features [S, 8] for records of the sets in CSR form.

    pix_of[s]: index (into `pixels`) of the output pixel of record s; ids, rho,
    colour per record; depth [N, H, W] float64 (as stored); frame f.
    """
    n_frames, h, w_img = depth.shape
    k = _poses.intrinsics(fx, fy, cx, cy)
    kinv = np.linalg.inv(k)
    s_count = ids.size
    out = np.zeros((s_count, N_FEAT))
    if s_count == 0:
        return out
    dj = (ids.astype(np.int64) >> _gather.ID_SHIFT) - window
    jj = f + dj
    q = (ids & ((1 << _gather.ID_SHIFT) - 1)).astype(np.int64)
    qx, qy = q % w_img, q // w_img
    counts = np.diff(offsets)
    med = lower_median(colour, offsets)
    pix = pixels[pix_of]
    x = (pix % w_img).astype(np.float64)
    y = (pix // w_img).astype(np.float64)
    dp = depth[f].reshape(-1)[pix]
    out[:, 0] = rho
    out[:, 1] = np.linalg.norm(colour - med[pix_of], axis=1)
    out[:, 2] = np.abs(dj) / window if window > 0 else 0.0
    out[:, 7] = dj / window if window > 0 else 0.0
    out[:, 6] = np.log1p(counts[pix_of]) / math.log1p((2 * radius + 1) ** 2 * (2 * window + 1))
    for j in np.unique(jj):
        sel = jj == j
        t = _poses.relative(cam_to_world[f], cam_to_world[j], same_frame=(j == f))
        u, v, z = _gather.project(dp[sel], x[sel], y[sel], t, k)
        out[sel, 3] = np.hypot(qx[sel] - u, qy[sel] - v)
        xf = dp[sel][None, :] * (kinv @ np.stack([x[sel], y[sel], np.ones(sel.sum())]))
        a = t[:3, :3] @ xf                     # X - o_f, in frame-J axes
        yj = a + t[:3, 3:4]                    # X - o_J
        out[sel, 4] = 1.0 - np.sum(a * yj, axis=0) / (np.linalg.norm(a, axis=0) * np.linalg.norm(yj, axis=0))
        out[sel, 5] = _depth_gradient(depth[j], qx[sel], qy[sel])
    return out


# ---------------------------------------------------------------------------
# forward, set softmax, loss, backward

def standardise(x: np.ndarray, mlp: MLP) -> np.ndarray:
    return (x - mlp.mean) / mlp.std


def forward(xs: np.ndarray, mlp: MLP):
    """Logits for standardised features xs [S, 8]; returns (m, cache)."""
    z1 = xs @ mlp.w1 + mlp.b1
    h1 = gelu(z1)
    z2 = h1 @ mlp.w2 + mlp.b2
    h2 = gelu(z2)
    m = h2 @ mlp.w3 + mlp.b3
    return m, (xs, z1, h1, z2, h2)


def set_softmax_mean(m: np.ndarray, colour: np.ndarray, offsets: np.ndarray, c_ref: np.ndarray):
    """O(p) = sum softmax(m)_s c_s per set (max-subtracted); empty set -> c_ref."""
    n = offsets.size - 1
    out = np.array(c_ref, dtype=np.float64, copy=True)
    a = np.zeros(m.size)
    for i in range(n):
        s, e = offsets[i], offsets[i + 1]
        if e > s:
            ex = np.exp(m[s:e] - m[s:e].max())
            a[s:e] = ex / ex.sum()
            out[i] = a[s:e] @ colour[s:e]
    return out, a


def loss_and_grads(xs, colour, offsets, c_ref, clean, mlp: MLP):
    """L = sum over non-empty sets of |O - G|^2, divided by 3 x (number of sets), and dL/dtheta."""
    m, (xs, z1, h1, z2, h2) = forward(xs, mlp)
    o, a = set_softmax_mean(m, colour, offsets, c_ref)
    counts = np.diff(offsets)
    used = counts > 0
    n_sets = max(counts.size, 1)
    diff = (o - clean) * used[:, None]
    loss = float(np.sum(diff * diff) / (3 * n_sets))
    d_o = 2.0 * diff / (3 * n_sets)
    seg = np.repeat(np.arange(counts.size), counts)
    # dO/dm_s = a_s (c_s - O)
    dm = a * np.sum((colour - o[seg]) * d_o[seg], axis=1)
    g = {}
    g["b3"] = float(dm.sum())
    g["w3"] = h2.T @ dm
    dz2 = np.outer(dm, mlp.w3) * gelu_grad(z2)
    g["w2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ mlp.w2.T) * gelu_grad(z1)
    g["w1"] = xs.T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, g, o


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0

    def __post_init__(self):
        self.m = {}
        self.v = {}

    def step(self, mlp: MLP, grads: dict) -> None:
        self.t += 1
        for name, gv in grads.items():
            gv = np.asarray(gv, dtype=np.float64)
            m = self.m.get(name, np.zeros_like(gv))
            v = self.v.get(name, np.zeros_like(gv))
            m = self.beta1 * m + (1 - self.beta1) * gv
            v = self.beta2 * v + (1 - self.beta2) * gv * gv
            self.m[name], self.v[name] = m, v
            mh = m / (1 - self.beta1 ** self.t)
            vh = v / (1 - self.beta2 ** self.t)
            upd = self.lr * mh / (np.sqrt(vh) + self.eps)
            cur = getattr(mlp, name)
            setattr(mlp, name, (cur - upd) if np.ndim(cur) else float(cur - upd))
