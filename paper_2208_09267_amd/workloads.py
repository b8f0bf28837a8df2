"""Seeded synthetic inputs of the VANSE lattice Boltzmann workloads.

This module holds input recipes only -- volume-fraction fields, initial
velocity fields and workload definitions -- and none of the method's
arithmetic.  Both the GPU path and the CPU oracle receive the arrays made
here.  It depends on numpy (and on torch for the *_device variants, which
evaluate the same recipes on the GPU for long request streams).

All fields are cell arrays with x fastest, cell = (z*ny + y)*nx + x, node
coordinates equal to the integer cell indices, periodic in every axis.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def grid(dims):
    """Integer node coordinates (x, y, z) broadcastable over [nz, ny, nx]."""
    nx, ny, nz = (list(dims) + [1, 1])[:3]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z


def channel_eps_2d(n=64, mean=0.8, amp=0.15):
    """phi(x, y, t) = mean + amp sin(2 pi x/n) cos(2 pi y/n) m(t): returns the
    static perturbation amp sin(2 pi x/n) cos(2 pi y/n) (the D2Q9 workload)."""
    x, y, _ = grid((n, n, 1))
    return (amp * np.sin(2 * np.pi * x / n) * np.cos(2 * np.pi * y / n)).ravel()


def fourier_eps(dims, seed, modes=8, kmax=4, amp=0.05, mean=0.75, lo=0.5, hi=1.0):
    """Seeded volume-fraction perturbation: a sum of `modes` random Fourier
    modes amp cos(2 pi k.x / N + theta) with integer wave vectors k in
    [-kmax, kmax]^3 \\ {0} and phases uniform in [0, 2 pi), added to `mean`,
    clipped to [lo, hi] and returned minus `mean`.  phi(x, t) = mean +
    m(t) * result stays in [lo, hi] for any |m| <= 1."""
    nx, ny, nz = (list(dims) + [1, 1])[:3]
    x, y, z = (np.arange(nx)[None, None, :], np.arange(ny)[None, :, None],
               np.arange(nz)[:, None, None])
    S = np.zeros((nz, ny, nx))
    for k, theta in fourier_modes(seed, modes, kmax):
        S += amp * np.cos(2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + theta)
    return (np.clip(mean + S, lo, hi) - mean).ravel()


def fourier_modes(seed, modes=8, kmax=4):
    """The (wave vector, phase) draws of fourier_eps for a seed."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(modes):
        k = rng.integers(-kmax, kmax + 1, 3)
        while not k.any():
            k = rng.integers(-kmax, kmax + 1, 3)
        out.append((k, rng.uniform(0.0, 2.0 * np.pi)))
    return out


def fourier_eps_device(dims, seed, device, modes=8, kmax=4, amp=0.05, mean=0.75, lo=0.5,
                       hi=1.0):
    """fourier_eps evaluated on a torch device (same draws, FP64; the values
    may differ from the numpy ones in the last bits).  For large request
    streams, where generating inputs on the host would dominate."""
    import torch

    nx, ny, nz = (list(dims) + [1, 1])[:3]
    x = torch.arange(nx, dtype=torch.float64, device=device).view(1, 1, nx)
    y = torch.arange(ny, dtype=torch.float64, device=device).view(1, ny, 1)
    z = torch.arange(nz, dtype=torch.float64, device=device).view(nz, 1, 1)
    S = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
    for k, theta in fourier_modes(seed, modes, kmax):
        S += amp * torch.cos(2 * np.pi * (float(k[0]) * x / nx + float(k[1]) * y / ny
                                          + float(k[2]) * z / nz) + theta)
    return (torch.clamp(mean + S, lo, hi) - mean).reshape(-1)


def taylor_green_device(dims, amp, device, d=3):
    """taylor_green on a torch device, SoA [d, ncells]."""
    import torch

    nx, ny, nz = (list(dims) + [1, 1])[:3]
    x = torch.arange(nx, dtype=torch.float64, device=device).view(1, 1, nx)
    y = torch.arange(ny, dtype=torch.float64, device=device).view(1, ny, 1)
    z = torch.arange(nz, dtype=torch.float64, device=device).view(nz, 1, 1)
    kx, ky, kz = 2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz
    ux = amp * torch.sin(kx * x) * torch.cos(ky * y) * torch.cos(kz * z)
    uy = -amp * torch.cos(kx * x) * torch.sin(ky * y) * torch.cos(kz * z)
    out = torch.zeros((d, nz * ny * nx), dtype=torch.float64, device=device)
    out[0] = ux.reshape(-1)
    out[1] = uy.reshape(-1)
    return out


def taylor_green(dims, amp):
    """Taylor-Green vortex u = amp (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0)
    with k = 2 pi / N per axis; returns SoA [3, ncells]."""
    nx, ny, nz = (list(dims) + [1, 1])[:3]
    x, y, z = grid(dims)
    kx, ky, kz = 2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz
    ux = amp * np.sin(kx * x) * np.cos(ky * y) * np.cos(kz * z)
    uy = -amp * np.cos(kx * x) * np.sin(ky * y) * np.cos(kz * z)
    return np.stack([ux.ravel(), uy.ravel(), np.zeros(ux.size)])


@dataclasses.dataclass
class Workload:
    """One solve: lattice, size, relaxation time, volume fraction and
    initial state.  phi(x, t_n) = eps_mean + cos(2 pi n / period) eps_pert."""
    name: str
    lattice: str            # "D2Q9" | "D3Q19"
    dims: tuple
    tau: float
    steps: int
    eps_mean: float
    period: float
    force: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    tgv_amp: float = 0.0
    quad_axes: int = 0

    @property
    def ncells(self):
        return int(np.prod(self.dims))

    def eps_pert(self):
        if self.lattice == "D2Q9":
            return channel_eps_2d(self.dims[0])
        return fourier_eps(self.dims, self.seed)

    def u0(self):
        d = 2 if self.lattice == "D2Q9" else 3
        if self.tgv_amp == 0.0:
            return np.zeros((d, self.ncells))
        return taylor_green(self.dims, self.tgv_amp)[:d]


def d2q9_64():
    """D2Q9, 64 x 64 periodic, tau 0.8, phi = 0.8 + 0.15 sin cos cos(2 pi t/2000),
    body force 1e-6 in x, rho 1, u 0, 1000 steps."""
    return Workload("D2Q9 64^2 tau=0.8", "D2Q9", (64, 64, 1), 0.8, 1000, 0.8, 2000.0,
                    force=(1e-6, 0.0, 0.0))


def d3q19_128():
    """D3Q19, 128^3, FP64, tau 0.6, 1000 steps, seeded Fourier phi (seed 1,
    period 1000 steps), Taylor-Green amplitude 0.02."""
    return Workload("D3Q19 128^3 tau=0.6", "D3Q19", (128, 128, 128), 0.6, 1000, 0.75, 1000.0,
                    seed=1, tgv_amp=0.02)


def d3q19_256():
    """D3Q19, 256^3, tau 0.55, 2000 steps, same phi construction (seed 1),
    Taylor-Green amplitude 0.02."""
    return Workload("D3Q19 256^3 tau=0.55", "D3Q19", (256, 256, 256), 0.55, 2000, 0.75, 1000.0,
                    seed=1, tgv_amp=0.02)


def batched_64(seed=3, count=64):
    """64 independent D3Q19 solves: edges uniform in {32, 48, 64, 96}, tau
    uniform in [0.55, 1.0], phi seeded 1000 + s, 500 steps each."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(rng.choice([32, 48, 64, 96]))
        tau = float(rng.uniform(0.55, 1.0))
        out.append(Workload("batch[%d] %d^3" % (s, n), "D3Q19", (n, n, n), tau, 500, 0.75,
                            1000.0, seed=1000 + s, tgv_amp=0.02))
    return out


def batched_256(seed=5, count=4):
    """`count` independent D3Q19 256^3 solves for the batched launch at the
    headline size: tau uniform in [0.55, 1.0], phi seeded 2000 + s,
    Taylor-Green amplitude 0.02, 200 steps each."""
    rng = np.random.default_rng(seed)
    return [Workload("batch256[%d]" % s, "D3Q19", (256, 256, 256), float(rng.uniform(0.55, 1.0)),
                     200, 0.75, 1000.0, seed=2000 + s, tgv_amp=0.02) for s in range(count)]


def served_arrivals(rate=20.0, duration=600.0, seed=4):
    """Poisson arrivals of D3Q19 requests: (arrival time, Workload).  Edge
    log-uniform in [32, 192], steps uniform in {500..5000}, tau uniform in
    [0.55, 1.0], phi seeded 100000 + r."""
    rng = np.random.default_rng(seed)
    t, r, out = 0.0, 0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        n = int(round(math.exp(rng.uniform(math.log(32), math.log(192)))))
        steps = int(rng.integers(500, 5001))
        tau = float(rng.uniform(0.55, 1.0))
        out.append((t, Workload("req[%d] %d^3" % (r, n), "D3Q19", (n, n, n), tau, steps, 0.75,
                                1000.0, seed=100000 + r, tgv_amp=0.02)))
        r += 1
