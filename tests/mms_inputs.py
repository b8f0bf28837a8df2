"""Inputs of the travelling manufactured-solution examples (Examples 3-5 of the
paper's numerical validation) evaluated with torch on any device.

Input generation only, no lattice Boltzmann arithmetic: it gives the volume
fraction phi, velocity u, pressure p and the manufactured force F_MMS at the
lattice nodes of the diffusively scaled set-up (2 m periodic box, rho = 1,
nu = 0.1 m^2/s, nodes at k dx), and the unit conversions.  The same arrays
feed the GPU run and the oracle's step in the parity tests.

With the active axes A (x; x, y; x, y, z), s_a = sin(pi (x_a - t/2)) and
c_a = cos(pi (x_a - t/2)):
  phi = 1/2 + 2/5 prod_a s_a,  p = prod_a s_a,  u_a = 1/2 + 1/phi (a in A).
Then phi u_a = phi/2 + 1 and phi u_a u_b = phi/4 + 1 + 1/phi, and since phi
travels at 1/2 along each active axis (d_t phi = -1/2 sum_b d_b phi) the
residual of the VANSE momentum equation reduces to
  F_a = -[a in A] (sum_b d_b phi)/phi^2 + phi d_a p
        + nu ( [a in A] (lap phi/phi - |grad phi|^2/phi^2)
               + sum_{b in A} (d_a d_b phi/phi - d_a phi d_b phi/phi^2) ).
"""
import math

import torch

NU = 0.1
L = 2.0


def setup(ex, N, tau):
    """(lattice name, dims, d, quad_axes, dx, dt, us, ps, fs) of Example ex
    (3, 4 or 5) at N nodes per active axis: velocity u_lu = u us, pressure
    p_lu = 1/3 + p ps, force F_lu = F fs."""
    if ex not in (3, 4, 5):
        raise ValueError("travelling examples are 3, 4 and 5")
    d = 3 if ex == 5 else 2
    dims = (N, 1 if ex == 3 else N, N if d == 3 else 1)
    quad = {3: 1, 4: 3, 5: 7}[ex]
    dx = L / N
    dt = (tau - 0.5) / 3.0 * dx * dx / NU
    return ("D3Q19" if d == 3 else "D2Q9"), dims, d, quad, dx, dt, dt / dx, (dt / dx) ** 2, \
        dt * dt / dx


def fields(ex, N, t, device="cpu"):
    """phi [n], u [3, n], p [n] and F_MMS [3, n] in physical units at time
    t, x fastest, as float64 tensors on `device`."""
    na = ex - 2
    dims = setup(ex, N, 0.6)[1]
    dx = L / N
    f64 = dict(dtype=torch.float64, device=device)
    s, c = [], []
    for a in range(3):
        if a < na:
            arg = math.pi * (torch.arange(dims[a], **f64) * dx - 0.5 * t)
            s.append(torch.sin(arg))
            c.append(torch.cos(arg))
        else:
            s.append(torch.ones(dims[a], **f64))
            c.append(torch.zeros(dims[a], **f64))

    def grid(vx, vy, vz):   # outer product, laid out [z][y][x]
        return (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).reshape(-1)

    P = grid(s[0], s[1], s[2])
    phi = 0.5 + 0.4 * P
    # first derivatives of P along each active axis, second derivatives of P
    dP = []
    for a in range(3):
        v = [s[0], s[1], s[2]]
        v[a] = math.pi * c[a]
        dP.append(grid(*v) if a < na else torch.zeros_like(P))
    d2P = [[None] * 3 for _ in range(3)]
    for a in range(3):
        for b in range(3):
            if a >= na or b >= na:
                d2P[a][b] = torch.zeros_like(P)
            elif a == b:
                d2P[a][b] = -math.pi * math.pi * P
            else:
                v = [s[0], s[1], s[2]]
                v[a] = math.pi * c[a]
                v[b] = math.pi * c[b]
                d2P[a][b] = grid(*v)
    dphi = [0.4 * q for q in dP]
    inv, inv2 = 1.0 / phi, 1.0 / (phi * phi)
    sum_dphi = sum(dphi[b] for b in range(na))
    lap = sum(0.4 * d2P[b][b] for b in range(na))
    grad2 = sum(dphi[b] * dphi[b] for b in range(na))
    u = torch.zeros(3, P.numel(), **f64)
    F = torch.zeros(3, P.numel(), **f64)
    for a in range(na):
        u[a] = 0.5 + inv
        visc = lap * inv - grad2 * inv2
        for b in range(na):
            visc = visc + 0.4 * d2P[a][b] * inv - dphi[a] * dphi[b] * inv2
        F[a] = -sum_dphi * inv2 + phi * dP[a] + NU * visc
    return phi, u, P, F
