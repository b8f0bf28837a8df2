"""Exact-arithmetic pin of whole oracle steps (CPU).

An independent transcription of the paper's time step in rational arithmetic
(fractions.Fraction), written from the equations and Tables 1-3, on tiny
periodic grids: the cell integral of the volume fraction (Laplacian form of
eq. quad, weights of Table 3), the central-difference gradient and the
pressure-correction force (eq. pressForce), the eps-weighted density and the
velocity with half the force (eqs. density, velocity), the equilibrium
(eq. feq, with rho*I = sum f) and Guo's forcing term in eq. lbe, then push
streaming.  Every input is an FP64 number taken exactly as a rational, so the
transcription computes the exact result of the oracle's own inputs; the
oracle's FP64 steps must agree to a few units in the last place on every
population.  The negative controls show that a dropped term, a wrong sign or
weight, or a transposed operand moves the exact result far outside that
tolerance.
"""
import itertools
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")
TABLES = json.load(open(GOLD))
LAT = {"D2Q9": (oracle.D2Q9, 2), "D3Q19": (oracle.D3Q19, 3), "D3Q27": (oracle.D3Q27, 3)}


def velocity_set(name):
    """{velocity vector (3-tuple): weight} from the paper's tables."""
    d = LAT[name][1]
    out = {}
    for g in TABLES[name]["groups"]:
        for v in itertools.product((-1, 0, 1), repeat=d):
            if sum(c * c for c in v) == g["norm2"]:
                out[tuple(v) + (0,) * (3 - d)] = Fr(g["weight"])
    return out


def exact_step(name, dims, tau, eps, f, fext, force, mistake=None):
    """One step in rational arithmetic.  eps[c], f[c][xi], force[a][c]; returns
    the new populations {(cell, xi): value}."""
    vs = velocity_set(name)
    d = LAT[name][1]
    nx, ny, nz = dims
    n_ax = d
    wq = Fr(TABLES["quadrature"][str(n_ax)]["wi"])
    if mistake == "weight":
        wq = wq * 2
    omega = 1 / tau

    def idx(x, y, z):
        return (x % nx) + nx * ((y % ny) + ny * (z % nz))

    out = {}
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        c = idx(x, y, z)
        e0 = eps[c]
        nb = []
        for a in range(d):
            step = [0, 0, 0]
            step[a] = 1
            ep = eps[idx(x + step[0], y + step[1], z + step[2])]
            em = eps[idx(x - step[0], y - step[1], z - step[2])]
            nb.append((ep, em))
        S = sum(ep + em for ep, em in nb)
        I = e0 + wq * (S - 2 * n_ax * e0)                         # cell integral
        g = [(ep - em) / 2 for ep, em in nb] + [Fr(0)] * (3 - d)  # central difference
        if mistake == "gradient_sign":
            g = [-v for v in g]
        M0 = sum(f[c][v] for v in vs)
        j = [sum(v[a] * f[c][v] for v in vs) for a in range(3)]
        rho = M0 / I                                              # eq. density
        p = rho / 3
        F = [fext[a] + p * g[a] + (force[a][c] if force is not None else 0) for a in range(3)]
        if mistake == "no_half_force":
            u = [j[a] / M0 for a in range(3)]
        else:
            u = [(j[a] + F[a] / 2) / M0 for a in range(3)]       # eq. velocity
        if mistake == "transposed":
            u = [u[1], u[0], u[2]]
        uu = sum(v * v for v in u)
        uF = sum(u[a] * F[a] for a in range(3))
        for v, w in vs.items():
            cu = sum(v[a] * u[a] for a in range(3))
            cF = sum(v[a] * F[a] for a in range(3))
            feq = w * M0 * (1 + 3 * cu + Fr(9, 2) * cu * cu - Fr(3, 2) * uu)
            guo = (1 - omega / 2) * w * (3 * (cF - uF) + 9 * cu * cF)
            post = f[c][v] - omega * (f[c][v] - feq) + guo
            out[(idx(x + v[0], y + v[1], z + v[2]), v)] = post    # push streaming
    return out


def _case(name, dims, seed, with_force):
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    lat, d = LAT[name]
    _, c_o, w_o = oracle.lattice(lat)
    eps = [rng.uniform(0.45, 0.95, n) for _ in range(2)]           # eps at t_0, t_1
    u0 = rng.uniform(-0.05, 0.05, (d, n))
    rho0 = rng.uniform(0.9, 1.1, n)
    f = oracle.init(lat, dims, eps[0], rho0, u0)
    f = f * (1 + rng.uniform(-0.02, 0.02, f.shape))                # off equilibrium
    fext = [float(v) for v in rng.uniform(-1e-3, 1e-3, 3)]
    if d == 2:
        fext[2] = 0.0
    force = None
    if with_force:
        force = rng.uniform(-1e-3, 1e-3, (3, n))
        if d == 2:
            force[2] = 0.0
    tau = float(rng.uniform(0.55, 1.4))
    return lat, c_o, eps, f, fext, force, tau


def _exact_inputs(c_o, eps, f, fext, force, tau, n):
    vecs = [tuple(int(a) for a in c) for c in c_o]
    fr_f = [{vecs[k]: Fr(float(f[c, k])) for k in range(len(vecs))} for c in range(n)]
    fr_eps = [Fr(float(v)) for v in eps]
    fr_fext = [Fr(v) for v in fext]
    fr_force = None if force is None else [[Fr(float(v)) for v in force[a]] for a in range(3)]
    return vecs, fr_f, fr_eps, fr_fext, fr_force, Fr(tau)


CASES = [("D2Q9", (3, 3, 1)), ("D2Q9", (4, 3, 1)), ("D3Q19", (3, 3, 3)), ("D3Q27", (3, 3, 3)),
         ("D3Q19", (2, 3, 4))]


@pytest.mark.parametrize("with_force", [False, True])
@pytest.mark.parametrize("name,dims", CASES)
def test_two_oracle_steps_equal_exact_arithmetic(name, dims, with_force):
    n = int(np.prod(dims))
    lat, c_o, eps, f, fext, force, tau = _case(name, dims, 11 + n, with_force)
    vecs, fr_f, fr_eps0, fr_fext, fr_force, fr_tau = _exact_inputs(c_o, eps[0], f, fext, force,
                                                                   tau, n)
    got = f
    exact = fr_f
    for k in range(2):
        got = oracle.step(lat, dims, tau, eps[k], got, force=force, fext=fext)
        fr_eps = [Fr(float(v)) for v in eps[k]]
        new = exact_step(name, dims, fr_tau, fr_eps, exact, fr_fext, fr_force)
        exact = [{v: new[(c, v)] for v in vecs} for c in range(n)]
    scale = max(abs(float(exact[c][v])) for c in range(n) for v in vecs)
    err = max(abs(got[c, k] - float(exact[c][vecs[k]])) for c in range(n) for k in range(len(vecs)))
    assert err <= 1e-14 * scale, err / scale


@pytest.mark.parametrize("mistake", ["weight", "gradient_sign", "no_half_force", "transposed"])
def test_exact_pin_detects_planted_mistakes(mistake):
    """Negative controls: the same comparison against a transcription with one
    planted mistake fails by many orders of magnitude more than the tolerance."""
    name, dims = "D3Q19", (3, 3, 3)
    n = 27
    lat, c_o, eps, f, fext, force, tau = _case(name, dims, 5, True)
    vecs, fr_f, fr_eps, fr_fext, fr_force, fr_tau = _exact_inputs(c_o, eps[0], f, fext, force,
                                                                  tau, n)
    got = oracle.step(lat, dims, tau, eps[0], f, force=force, fext=fext)
    new = exact_step(name, dims, fr_tau, fr_eps, fr_f, fr_fext, fr_force, mistake=mistake)
    scale = max(abs(float(v)) for v in new.values())
    err = max(abs(got[c, k] - float(new[(c, vecs[k])])) for c in range(n) for k in range(len(vecs)))
    assert err > 1e-9 * scale, (mistake, err / scale)
