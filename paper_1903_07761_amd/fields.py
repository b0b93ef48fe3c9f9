"""Seeded synthetic scalar fields standing in for the paper's datasets.

The paper compresses Cubism-MPCF snapshots of cavitating bubble clouds (Sec.
3.1: a cloud of log-normally sized bubbles in a cubic domain, fields p, rho, E,
alpha_2 on 512^3 and 1024^3 grids of 32^3 blocks).  Those files are not
available, so these generators produce fields of the same shapes and
structure.  This module holds none of the wavelet arithmetic: it only makes
inputs, and serves both the GPU path and the CPU oracle.

All random draws come from numpy ``Generator(PCG64(seed))`` in a fixed order;
the deterministic math runs in float64 with torch on the requested device and
is cast to the requested dtype at the end.  Coordinates are cell centres
x_i = (i + 1/2) / n of the unit box; arrays are indexed [z, y, x].

G1 ``gaussian_bumps``: 8 bumps (cx, cy, cz ~ U[0,1), sigma ~ U(0.05, 0.2),
    A ~ U(0.5, 2), drawn in that order per bump) plus
    0.1 sin(2 pi x) cos(2 pi y).
G2 ``bubble_cloud``: B bubbles (centre ~ U[0,1)^3, radius =
    exp(N(ln 0.02, 0.4))); phi = min_b (|x - c_b| - r_b);
    H = (1 + tanh(phi / delta)) / 2 with delta = 2 / n (two cells);
    v = v_in + (v_out - v_in) H; then v *= 1 + noise * xi, xi ~ N(0, 1) drawn
    as one C-order n^3 array after the geometry.  Pressure-like: v_in 0.1,
    v_out 1.0; density-like: v_in 0.016, v_out 1.0 (the paper's rho min/max
    ratio, Table 1).
G3 ``div_free_velocity``: u = (0.1 / M) sum_m a_m cos(2 pi k_m . x + theta_m),
    M = 8, k_m in {-4..4}^3 \\ {0}, a_m = unit(g - (g . k^) k^) with
    g ~ N(0, I), theta_m ~ U[0, 2 pi); div u = 0 exactly.
"""
from __future__ import annotations

import math

import numpy as np
import torch

_TANH_SATURATED = 40.0  # tanh(t) == 1.0 in float64 for t >= 40 (|1 - tanh| < 1e-34)


def _coords(n: int, device) -> torch.Tensor:
    return (torch.arange(n, device=device, dtype=torch.float64) + 0.5) / n


def _z_chunks(n: int, budget_points: int = 1 << 25):
    step = max(1, budget_points // (n * n))
    for z0 in range(0, n, step):
        yield z0, min(n, z0 + step)


def gaussian_bumps(n: int, seed: int, *, dtype=torch.float32, device="cpu", nbumps: int = 8) -> torch.Tensor:
    rng = np.random.Generator(np.random.PCG64(seed))
    bumps = []
    for _ in range(nbumps):
        cx, cy, cz = rng.uniform(0.0, 1.0, 3)
        sigma = rng.uniform(0.05, 0.2)
        amp = rng.uniform(0.5, 2.0)
        bumps.append((cx, cy, cz, sigma, amp))
    x = _coords(n, device)
    out = torch.empty((n, n, n), dtype=dtype, device=device)
    base_xy = 0.1 * torch.sin(2 * math.pi * x)[None, :] * torch.cos(2 * math.pi * x)[:, None]  # [y, x]
    for z0, z1 in _z_chunks(n):
        z = x[z0:z1]
        f = base_xy[None].expand(z1 - z0, n, n).clone()
        for cx, cy, cz, sigma, amp in bumps:
            r2 = ((z - cz) ** 2)[:, None, None] + ((x - cy) ** 2)[None, :, None] + ((x - cx) ** 2)[None, None, :]
            f += amp * torch.exp(-r2 / (2 * sigma * sigma))
        out[z0:z1] = f.to(dtype)
    return out


def draw_bubbles(seed: int, nbubbles: int = 200):
    """Centres [B, 3] (x, y, z) and radii [B] of a seeded bubble cloud, and the
    generator positioned after those draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = np.empty((nbubbles, 3))
    radii = np.empty(nbubbles)
    for b in range(nbubbles):
        centres[b] = rng.uniform(0.0, 1.0, 3)
        radii[b] = math.exp(rng.normal(math.log(0.02), 0.4))
    return centres, radii, rng


def bubble_cloud(n: int, seed: int, *, nbubbles: int = 200, v_in: float = 0.1, v_out: float = 1.0,
                 noise: float = 0.01, noise_seed: int | None = None, dtype=torch.float32,
                 device="cpu") -> torch.Tensor:
    centres, radii, nrng = draw_bubbles(seed, nbubbles)
    if noise_seed is not None:  # same bubbles, independent noise (e.g. rho beside p)
        nrng = np.random.Generator(np.random.PCG64(noise_seed))
    delta = 2.0 / n
    cutoff = _TANH_SATURATED * delta
    x = _coords(n, device)
    cz_all = torch.tensor(centres, dtype=torch.float64, device=device)
    r_all = torch.tensor(radii, dtype=torch.float64, device=device)
    out = torch.empty((n, n, n), dtype=dtype, device=device)
    for z0, z1 in _z_chunks(n):
        zlo, zhi = (z0 + 0.5) / n, (z1 - 0.5) / n
        # bubbles that can bring phi below the tanh saturation in this slab; the
        # others cannot change H (exactly 1 there), so skipping them is exact.
        gap = np.maximum(0.0, np.maximum(zlo - centres[:, 2], centres[:, 2] - zhi))
        near = np.nonzero(gap < radii + cutoff)[0]
        z = x[z0:z1]
        phi = torch.full((z1 - z0, n, n), cutoff * 2, dtype=torch.float64, device=device)
        for b in near.tolist():
            cx, cy, cz = cz_all[b, 0], cz_all[b, 1], cz_all[b, 2]
            d = torch.sqrt(((z - cz) ** 2)[:, None, None] + ((x - cy) ** 2)[None, :, None]
                           + ((x - cx) ** 2)[None, None, :]) - r_all[b]
            torch.minimum(phi, d, out=phi)
        H = 0.5 * (1.0 + torch.tanh(phi / delta))
        v = v_in + (v_out - v_in) * H
        if noise:
            xi = torch.from_numpy(nrng.standard_normal((z1 - z0) * n * n)).to(device).view(z1 - z0, n, n)
            v = v * (1.0 + noise * xi)
        out[z0:z1] = v.to(dtype)
    return out


def div_free_velocity(n: int, seed: int, *, modes: int = 8, amplitude: float = 0.1, dtype=torch.float32,
                      device="cpu"):
    """Three components (u, v, w) of a divergence-free sinusoid sum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    waves = []
    while len(waves) < modes:
        k = rng.integers(-4, 5, 3)
        if not k.any():
            continue
        g = rng.standard_normal(3)
        khat = k / np.linalg.norm(k)
        a = g - (g @ khat) * khat
        a /= np.linalg.norm(a)
        theta = rng.uniform(0.0, 2 * math.pi)
        waves.append((k.astype(np.float64), a, theta))
    x = _coords(n, device)
    comps = [torch.empty((n, n, n), dtype=dtype, device=device) for _ in range(3)]
    for z0, z1 in _z_chunks(n):
        z = x[z0:z1]
        acc = [torch.zeros((z1 - z0, n, n), dtype=torch.float64, device=device) for _ in range(3)]
        for k, a, theta in waves:
            ph = (2 * math.pi) * (k[2] * z[:, None, None] + k[1] * x[None, :, None] + k[0] * x[None, None, :]) + theta
            c = torch.cos(ph)
            for i in range(3):
                acc[i] += a[i] * c
        for i in range(3):
            comps[i][z0:z1] = ((amplitude / modes) * acc[i]).to(dtype)
    return comps


def value_range(field: torch.Tensor) -> float:
    return float(field.max().item()) - float(field.min().item())
