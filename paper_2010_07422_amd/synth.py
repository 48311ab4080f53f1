"""Seeded synthetic inputs for IRCUR runs, tests and benchmarks.

This module only generates data; it holds none of the method's arithmetic, and
both the oracle-side tests and the GPU path draw their inputs from it.

Workloads (all NumPy, float64 unless stated):

* ``planted`` -- the synthetic RPCA instance of the paper's supplementary
  setup: L = W V^T with W, V i.i.d. N(0, 1) of shape n x r; S with an exactly
  round(alpha n1 n2) uniformly drawn support and i.i.d. values uniform in
  [-c E|L_ij|, c E|L_ij|] (E|L_ij| taken as the empirical mean over all
  entries; the paper uses c = 1, the configurations here use c = 10).
* ``video`` -- a stand-in for the surveillance-video benchmark (frames as
  columns): a rank-2 smooth background field times slowly varying per-frame
  gains, plus four rectangular blobs moving linearly.
* ``unrolled_batch`` -- the ragged batch for the unrolled, differentiable mode.
* ``planted_device`` -- the planted recipe drawn with torch on a device (for
  sweeps at sizes where generating on the host is slow); same laws, its own
  random stream.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Planted:
    D: np.ndarray          # (n1, n2) float64, D = L + S
    W: np.ndarray          # (n1, r)  L = W @ V.T
    V: np.ndarray          # (n2, r)
    support: np.ndarray    # flat indices of the outliers
    values: np.ndarray     # outlier values
    r: int
    alpha: float

    @property
    def L(self) -> np.ndarray:
        return self.W @ self.V.T

    @property
    def Lmax(self) -> float:
        return float(np.abs(self.W @ self.V.T).max())


def planted(n1: int, n2: int, r: int, alpha: float, seed: int,
            outlier_scale: float = 10.0, rank_true: int | None = None) -> Planted:
    """Planted low-rank plus sparse instance (seeded)."""
    rng = np.random.default_rng(seed)
    rt = r if rank_true is None else rank_true
    W = rng.standard_normal((n1, rt))
    V = rng.standard_normal((n2, rt))
    L = W @ V.T
    mean_abs = float(np.abs(L).mean())
    k = int(round(alpha * n1 * n2))
    support = rng.choice(n1 * n2, size=k, replace=False) if k > 0 else np.zeros(0, np.int64)
    c = outlier_scale * mean_abs
    values = rng.uniform(-c, c, size=k)
    D = L
    D.reshape(-1)[support] += values
    return Planted(D=D, W=W, V=V, support=support, values=values, r=rt, alpha=alpha)


def exact_lowrank(n1: int, n2: int, r: int, seed: int):
    """Exactly rank-r D = W V^T with no outliers; returns (D, W, V)."""
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((n1, r))
    V = rng.standard_normal((n2, r))
    return W @ V.T, W, V


def _smooth_field(rng, h, w, sigma):
    from scipy.ndimage import gaussian_filter
    f = gaussian_filter(rng.standard_normal((h, w)), sigma=sigma, mode="wrap")
    f -= f.min()
    f /= max(f.max(), 1e-300)
    return f


@dataclass
class Video:
    D: np.ndarray          # (h*w, frames) float32 or float64
    F: np.ndarray          # (h*w, 2) background fields
    G: np.ndarray          # (frames, 2) per-frame gains; L = F @ G.T
    fg_density: float      # realised fraction of nonzero foreground entries


def video(h: int = 240, w: int = 320, frames: int = 1200, seed: int = 3,
          nblobs: int = 4, blob_hw=(20, 30), dtype=np.float32) -> Video:
    """Video-shaped instance: columns are vectorised frames (pixels x frames)."""
    rng = np.random.default_rng(seed)
    f1 = _smooth_field(rng, h, w, sigma=24.0).reshape(-1)
    f2 = _smooth_field(rng, h, w, sigma=12.0).reshape(-1)
    t = np.arange(frames, dtype=np.float64)
    g1 = 0.8 + 0.2 * np.sin(2.0 * math.pi * t / frames)
    g2 = 0.1 * t / max(frames - 1, 1)
    F = np.stack([f1, f2], axis=1)
    G = np.stack([g1, g2], axis=1)
    D = (F @ G.T).astype(dtype)
    bh, bw = blob_hw
    nnz = 0
    for _ in range(nblobs):
        y0, x0 = rng.uniform(0, h - bh), rng.uniform(0, w - bw)
        y1, x1 = rng.uniform(0, h - bh), rng.uniform(0, w - bw)
        inten = rng.uniform(0.5, 1.0)
        for fr in range(frames):
            a = fr / max(frames - 1, 1)
            y = int(round(y0 + a * (y1 - y0)))
            x = int(round(x0 + a * (x1 - x0)))
            rows = (np.arange(y, y + bh)[:, None] * w + np.arange(x, x + bw)[None, :]).reshape(-1)
            D[rows, fr] += dtype(inten)
            nnz += rows.size
    return Video(D=D, F=F, G=G, fg_density=nnz / D.size)


@dataclass
class BatchItem:
    inst: Planted
    n: int
    s: int


def unrolled_batch(nb: int = 32, nmin: int = 1000, nmax: int = 3000, r: int = 5,
                   amin: float = 0.1, amax: float = 0.3, c: float = 4.0,
                   seed: int = 7) -> list:
    """Ragged batch of planted instances, n_b ~ U{nmin..nmax}, alpha_b ~ U[amin, amax]."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(nb):
        n = int(rng.integers(nmin, nmax + 1))
        a = float(rng.uniform(amin, amax))
        inst = planted(n, n, r, a, seed=int(rng.integers(0, 2**31 - 1)))
        out.append(BatchItem(inst=inst, n=n, s=int(math.ceil(c * r * math.log(n)))))
    return out


def sample_size(c: float, r: int, n: int) -> int:
    """ceil(c r ln n) rows or columns (the sampling rule of the paper)."""
    return int(math.ceil(c * r * math.log(n)))


# Named workloads.  Each entry fixes the generator arguments and the solver
# parameters; "s" is |I| = |J| unless sI/sJ are given.
CONFIGS = {
    "planted_n1000_r5_f64": dict(kind="planted", n=1000, r=5, alpha=0.1, c=4.0,
                                 dtype="f64", gamma=0.7, eps=0.0, max_iter=30,
                                 data_seed=0, index_seed=1, resample=True),
    "planted_n3000_r5_f32": dict(kind="planted", n=3000, r=5, alpha=0.2, c=4.0,
                                 dtype="f32", gamma=0.7, eps=1e-5, max_iter=100,
                                 data_seed=0, index_seed=1, resample=True),
    "planted_n10000_r10_bf16": dict(kind="planted", n=10000, r=10, alpha=0.3, c=3.0,
                                    dtype="bf16", gamma=0.7, eps=1e-5, max_iter=100,
                                    data_seed=0, index_seed=1, resample=True),
    "video_76800x1200_r2_f32": dict(kind="video", h=240, w=320, frames=1200, r=2,
                                    sI=800, sJ=200, dtype="f32", gamma=0.7,
                                    eps=1e-5, max_iter=100, data_seed=3,
                                    index_seed=1, resample=True),
}


@dataclass
class PlantedDevice:
    D: "object"            # (n1, n2) torch tensor of the requested dtype
    W: "object"            # (n1, r) float64, L = W @ V.T
    V: "object"            # (n2, r) float64
    nnz: int               # outliers drawn: round(alpha n1 n2)
    Lmax: float            # max |L_ij|
    mean_abs: float        # mean |L_ij|


def planted_device(n1: int, n2: int, r: int, alpha: float, seed: int, device="cuda",
                   dtype=None, outlier_scale: float = 10.0, row_block: int = 4096) -> PlantedDevice:
    """The planted recipe of ``planted`` drawn with a seeded torch generator
    on `device`: W, V i.i.d. N(0, 1); exactly round(alpha n1 n2) outlier
    positions drawn without replacement; values uniform in +-outlier_scale
    mean|L|.  L is formed in row blocks so that only D is held whole."""
    import torch
    dtype = torch.float64 if dtype is None else dtype
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    W = torch.randn((n1, r), generator=g, device=device, dtype=torch.float64)
    V = torch.randn((n2, r), generator=g, device=device, dtype=torch.float64)
    D = torch.empty((n1, n2), device=device, dtype=dtype)
    lmax, lsum = 0.0, 0.0
    for i0 in range(0, n1, row_block):
        Lb = W[i0:i0 + row_block] @ V.T
        lmax = max(lmax, float(Lb.abs().max()))
        lsum += float(Lb.abs().sum())
        D[i0:i0 + row_block] = Lb.to(dtype)
    mean_abs = lsum / (n1 * n2)
    k = int(round(alpha * n1 * n2))
    if k > 0:
        pos = torch.randperm(n1 * n2, generator=g, device=device)[:k]
        c = outlier_scale * mean_abs
        vals = (torch.rand(k, generator=g, device=device, dtype=torch.float64) * 2.0 - 1.0) * c
        flat = D.view(-1)
        for j0 in range(0, k, 1 << 26):
            pj = pos[j0:j0 + (1 << 26)]
            rows = torch.div(pj, n2, rounding_mode="floor")
            Lv = (W[rows] * V[pj - rows * n2]).sum(1)
            flat[pj] = (Lv + vals[j0:j0 + (1 << 26)]).to(dtype)
        del pos, vals
    return PlantedDevice(D=D, W=W, V=V, nnz=k, Lmax=lmax, mean_abs=mean_abs)
