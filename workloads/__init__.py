"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds none of the method's arithmetic: it only evaluates input
surface densities at points it is given (the sample lattice comes from
whichever side is being tested) and draws seeded random parameters.

Workloads (all synthetic; the paper uses no dataset):

* generalised Maclaurin disks D_n (Sec. 3): sigma0 (1 - R^2/a^2)^(n - 1/2)
  for R < a, else 0;
* Gaussian clumps: sum_c a_c exp(-|x - x_c|^2 / (2 s_c^2)) times the taper
  (1 - (r/0.95)^2)^4 for r < 0.95 (0 beyond), a_c ~ U(0.1, 1),
  s_c ~ U(0.02, 0.1), centres area-uniform in r <= 0.85
  (r = 0.85 sqrt(u), theta = 2 pi v), drawn from numpy's PCG64
  ``default_rng(seed)`` in the order a, s, u, v;
* sparse coefficient sets (a few seeded impulses) whose forces an exact
  superposition can check at any grid size;
* batches of disks of mixed sizes and orders: n ~ U{96, 128, 192, 256, 384,
  512, 768, 1024, 1536, 2048}, k ~ U{1, 2, 3}, clump count ~ U{4..64}, all
  from ``default_rng(seed)`` in that order, each disk's clumps from the
  children of ``SeedSequence(seed)``.
"""
from __future__ import annotations

import numpy as np


def disk_sigma(n: int, alpha: float, xs: np.ndarray, ys: np.ndarray, sigma0: float = 1.0) -> np.ndarray:
    """D_n surface density on the tensor lattice (xs, ys); result [len(ys)][len(xs)]."""
    X, Y = np.meshgrid(np.asarray(xs, np.float64), np.asarray(ys, np.float64))
    u = 1.0 - (X * X + Y * Y) / (alpha * alpha)
    return np.where(u > 0, sigma0 * np.power(np.maximum(u, 0.0), n - 0.5), 0.0)


def clump_params(seed, n_clumps: int):
    """Seeded clump parameters (amplitude, width, centre x, centre y)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.1, 1.0, n_clumps)
    s = rng.uniform(0.02, 0.1, n_clumps)
    u = rng.uniform(0.0, 1.0, n_clumps)
    v = rng.uniform(0.0, 1.0, n_clumps)
    r = 0.85 * np.sqrt(u)
    th = 2.0 * np.pi * v
    return a, s, r * np.cos(th), r * np.sin(th)


def clump_sigma(params, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Tapered sum of Gaussian clumps on the lattice (xs, ys)."""
    a, s, cx, cy = params
    xs = np.asarray(xs, np.float64)
    ys = np.asarray(ys, np.float64)
    out = np.zeros((ys.size, xs.size))
    for c in range(len(a)):
        gx = np.exp(-(xs - cx[c]) ** 2 / (2.0 * s[c] ** 2))
        gy = np.exp(-(ys - cy[c]) ** 2 / (2.0 * s[c] ** 2))
        out += a[c] * np.outer(gy, gx)
    X, Y = np.meshgrid(xs, ys)
    rr = np.sqrt(X * X + Y * Y) / 0.95
    taper = np.where(rr < 1.0, np.power(np.maximum(1.0 - rr * rr, 0.0), 4), 0.0)
    return out * taper


def perturb_clumps(params, seed, amp_frac: float = 0.1, shift: float = 0.01):
    """Seeded perturbation of clump parameters (target densities for a
    fitting loss): a_c (1 + amp_frac xi), x_c + shift eta, xi, eta ~ N(0, 1)."""
    a, s, cx, cy = params
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(len(a))
    ex = rng.standard_normal(len(a))
    ey = rng.standard_normal(len(a))
    return a * (1.0 + amp_frac * xi), s, cx + shift * ex, cy + shift * ey


def sparse_coeffs(seed, M: int, N: int, count: int, margin: int = 0):
    """``count`` seeded impulse positions (i, j) and values in [-1, 1]."""
    rng = np.random.default_rng(seed)
    i = rng.integers(margin, M - margin, count).astype(np.int32)
    j = rng.integers(margin, N - margin, count).astype(np.int32)
    c = rng.uniform(-1.0, 1.0, count)
    return i, j, c


def sample_cells(seed, M: int, N: int, count: int, extra=()):
    """Seeded flat cell indices j*M + i (plus any ``extra`` ones), unique."""
    rng = np.random.default_rng(seed)
    cells = rng.integers(0, M * N, count).astype(np.int64)
    border = [0, M - 1, (N - 1) * M, N * M - 1]
    return np.unique(np.concatenate([cells, np.asarray(border + list(extra), np.int64)]))


BATCH_SIZES = (96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048)


def batch_disks(seed=4, count=256):
    """[(n, k, clump parameters), ...] for a seeded batch of square disks on [-1,1]^2."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.array(BATCH_SIZES), count)
    k = rng.integers(1, 4, count)
    nc = rng.integers(4, 65, count)
    children = np.random.SeedSequence(seed).spawn(count)
    return [(int(n[i]), int(k[i]), clump_params(children[i], int(nc[i]))) for i in range(count)]


def clump_sigma_torch(params, xs, ys, device="cuda"):
    """clump_sigma evaluated with torch on a device (float64)."""
    import torch
    a, s, cx, cy = (torch.as_tensor(np.asarray(v, np.float64), device=device) for v in params)
    x = torch.as_tensor(np.asarray(xs, np.float64), device=device)
    y = torch.as_tensor(np.asarray(ys, np.float64), device=device)
    gx = torch.exp(-(x[None, :] - cx[:, None]) ** 2 / (2.0 * s[:, None] ** 2))     # [c][nx]
    gy = torch.exp(-(y[None, :] - cy[:, None]) ** 2 / (2.0 * s[:, None] ** 2))     # [c][ny]
    out = (gy * a[:, None]).transpose(0, 1).contiguous() @ gx.contiguous()           # [ny][nx]
    X, Y = x[None, :], y[:, None]
    rr = torch.sqrt(X * X + Y * Y) / 0.95
    taper = torch.where(rr < 1.0, torch.clamp(1.0 - rr * rr, min=0.0) ** 4, torch.zeros_like(rr))
    return out * taper
