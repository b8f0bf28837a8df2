"""Pins of the oracle's constant tables and volume-fraction operators.

Lattice tables: Tables 1-2 of the paper (golden fixture) and the exact
isotropy identities that make c_s^2 = 1/3.  Quadrature weights: Table 3 and
the equality of the two printed forms of the cell integral (eq. quad, the
weighted sum over neighbours, and eq. latDiffRuleIIre, the Laplacian form).
Gradient: the central difference formula of the pressure-correction section.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
NAMES = {oracle.D2Q9: "D2Q9", oracle.D3Q19: "D3Q19", oracle.D3Q27: "D3Q27"}


@pytest.mark.parametrize("lat", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
def test_lattice_matches_paper_tables(lat):
    d, c, w = oracle.lattice(lat)
    groups = GOLD[NAMES[lat]]["groups"]
    assert len(c) == sum(g["count"] for g in groups)
    norms = (c ** 2).sum(1)
    for g in groups:
        sel = norms == g["norm2"]
        assert sel.sum() == g["count"]
        assert np.all(w[sel] == float(Fraction(g["weight"])))
    # every velocity appears once and its opposite is present
    assert len({tuple(v) for v in c}) == len(c)
    for v in c:
        assert any((u == -v).all() for u in c)
    assert np.all(np.abs(c) <= 1)
    if d == 2:
        assert np.all(c[:, 2] == 0)


@pytest.mark.parametrize("lat", [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27])
def test_lattice_isotropy_gives_cs2_one_third(lat):
    d, c, w = oracle.lattice(lat)
    wf = [Fraction(x).limit_denominator(1000) for x in w]
    assert sum(wf) == 1
    for a in range(d):
        assert sum(wi * int(ci[a]) for wi, ci in zip(wf, c)) == 0
        for b in range(d):
            m2 = sum(wi * int(ci[a]) * int(ci[b]) for wi, ci in zip(wf, c))
            assert m2 == (Fraction(1, 3) if a == b else 0)
    # fourth-order isotropy: sum w xa xb xc xd = (dab dcd + dac dbd + dad dbc)/9
    rng = range(d)
    for a in rng:
        for b in rng:
            for e in rng:
                for g in rng:
                    m4 = sum(wi * int(ci[a] * ci[b] * ci[e] * ci[g]) for wi, ci in zip(wf, c))
                    want = Fraction(int(a == b and e == g) + int(a == e and b == g)
                                    + int(a == g and b == e), 9)
                    assert m4 == want


@pytest.mark.parametrize("n", [1, 2, 3])
def test_quadrature_weights_table3(n):
    w0, wi = oracle.quad_weights(n)
    gold = GOLD["quadrature"][str(n)]
    assert w0 == float(Fraction(gold["w0"]))
    assert wi == float(Fraction(gold["wi"]))
    # a quadrature of a constant must return the constant
    assert Fraction(gold["w0"]) + 2 * n * Fraction(gold["wi"]) == 1


def _random_state(lat, dims, seed):
    rng = np.random.default_rng(seed)
    n = oracle.ncells(dims)
    eps = rng.uniform(0.3, 1.0, n)
    d = 2 if lat == oracle.D2Q9 else 3
    u0 = rng.uniform(-0.05, 0.05, (d, n))
    rho0 = rng.uniform(0.9, 1.1, n)
    f = oracle.init(lat, dims, eps, rho0, u0)
    f = f * rng.uniform(0.97, 1.03, f.shape)  # leave equilibrium
    return eps, f


def _shift(a, dims, axis, s):
    nx, ny, nz = (list(dims) + [1, 1])[:3]
    return np.roll(a.reshape(nz, ny, nx), -s, axis=2 - axis).ravel()


@pytest.mark.parametrize("lat,dims,mask", [
    (oracle.D2Q9, (7, 5), 3), (oracle.D2Q9, (6, 4), 1), (oracle.D2Q9, (6, 4), 2),
    (oracle.D3Q19, (5, 4, 3), 7), (oracle.D3Q19, (5, 4, 3), 5), (oracle.D3Q27, (4, 3, 5), 7),
    (oracle.D3Q19, (4, 4, 4), 1)])
def test_cell_integral_equals_weighted_neighbour_sum(lat, dims, mask):
    """rho = M0 / I with I = sum_i varpi_i phi(x - xi_i) over the D1Q3/D2Q5/D3Q7
    stencil of the quadrature axes (eq. quad, Table 3)."""
    eps, f = _random_state(lat, dims, 11)
    rho, _, _ = oracle.moments(lat, dims, eps, f, quad_axes=mask)
    M0 = f.sum(1)
    n_axes = bin(mask).count("1")
    gold = GOLD["quadrature"][str(n_axes)]
    w0, wi = float(Fraction(gold["w0"])), float(Fraction(gold["wi"]))
    I = w0 * eps
    for a in range(3):
        if mask & (1 << a):
            I = I + wi * (_shift(eps, dims, a, 1) + _shift(eps, dims, a, -1))
    np.testing.assert_allclose(M0 / rho, I, rtol=1e-14, atol=0)


@pytest.mark.parametrize("lat,dims", [(oracle.D2Q9, (7, 5)), (oracle.D3Q19, (5, 4, 3)),
                                      (oracle.D3Q27, (3, 4, 5))])
def test_pressure_correction_force_is_p_central_gradient(lat, dims):
    """F = p grad(phi) + F_ext with grad by central differences (eq. pressForce)
    and u = (j + F/2)/M0 (eq. velocity): recover F from the moments."""
    d, c, w = oracle.lattice(lat)
    eps, f = _random_state(lat, dims, 5)
    fext = np.array([1e-3, -2e-3, 5e-4])
    rho, p, u = oracle.moments(lat, dims, eps, f, fext=fext)
    M0 = f.sum(1)
    j = f @ c[:, :d]
    F = 2.0 * (u.T * M0[:, None] - j)
    for a in range(d):
        grad = 0.5 * (_shift(eps, dims, a, 1) - _shift(eps, dims, a, -1))
        np.testing.assert_allclose(F[:, a], p * grad + fext[a], rtol=1e-10, atol=1e-15)
    np.testing.assert_allclose(p, rho / 3.0, rtol=1e-15)


def test_eps_one_gives_unit_integral_exactly():
    """With phi == 1 the Laplacian form gives I = 1 exactly (the weighted-sum
    form would round to 1 - 2^-53 for D2Q5)."""
    for lat, dims in [(oracle.D2Q9, (4, 3)), (oracle.D3Q19, (3, 3, 3))]:
        n = oracle.ncells(dims)
        eps = np.ones(n)
        _, f = _random_state(lat, dims, 2)
        rho, _, _ = oracle.moments(lat, dims, eps, f)
        M0 = np.zeros(n)
        for i in range(f.shape[1]):  # the oracle's summation order
            M0 = M0 + f[:, i]
        assert np.array_equal(rho, M0)
