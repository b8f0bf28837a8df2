"""Pins of the oracle's collision and full time step.

  * equilibrium moments (eqs. M0-M2 with rho * I = M0) and forcing moments
    (eqs. M0F-M2F of the Chapman-Enskog appendix) on random inputs;
  * the BGK + Guo step against an independent textbook formulation
    (Krueger et al. 2017, eqs. 3.54 and 6.14 in vector form);
  * phi == 1 reduces the VANSE step to that BGK step bit for bit;
  * phi == const: homogeneity (f halves exactly when phi and F halve);
  * conservation: sum_x M0 constant; momentum gains sum_x F per step;
  * translation covariance on a periodic lattice;
  * the shear viscosity nu = (tau - 1/2) c_s^2 of the appendix.
"""
import numpy as np
import pytest

import oracle

LATS = [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27]


def _d(lat):
    return 2 if lat == oracle.D2Q9 else 3


@pytest.mark.parametrize("lat", LATS)
def test_equilibrium_moments(lat):
    d, c, w = oracle.lattice(lat)
    rng = np.random.default_rng(lat)
    for _ in range(20):
        M0 = rng.uniform(0.2, 1.5)
        u = np.zeros(3)
        u[:d] = rng.uniform(-0.1, 0.1, d)
        fe = oracle.feq(lat, M0, u)
        cc = c[:, :d].astype(float)
        np.testing.assert_allclose(fe.sum(), M0, rtol=1e-14)
        np.testing.assert_allclose(cc.T @ fe, M0 * u[:d], rtol=1e-13, atol=1e-16)
        second = np.einsum("ia,ib,i->ab", cc, cc, fe)
        want = M0 * (np.outer(u[:d], u[:d]) + np.eye(d) / 3.0)
        np.testing.assert_allclose(second, want, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("lat", LATS)
def test_forcing_moments(lat):
    d, c, w = oracle.lattice(lat)
    rng = np.random.default_rng(10 + lat)
    for _ in range(20):
        tau = rng.uniform(0.51, 2.0)
        u = np.zeros(3)
        F = np.zeros(3)
        u[:d] = rng.uniform(-0.1, 0.1, d)
        F[:d] = rng.uniform(-1e-3, 1e-3, d)
        om = oracle.forcing(lat, tau, u, F)
        k = 1.0 - 0.5 / tau
        cc = c[:, :d].astype(float)
        assert abs(om.sum()) < 1e-18
        np.testing.assert_allclose(cc.T @ om, k * F[:d], rtol=1e-12, atol=1e-19)
        second = np.einsum("ia,ib,i->ab", cc, cc, om)
        want = k * (np.outer(F[:d], u[:d]) + np.outer(u[:d], F[:d]))
        np.testing.assert_allclose(second, want, rtol=1e-11, atol=1e-19)


def _textbook_bgk_guo(lat, dims, tau, f, fext):
    """Independent numpy formulation of one BGK step with Guo forcing:
    rho = sum f, u = (sum xi f + F/2)/rho,
    feq = w rho [1 + xi.u/cs2 + (xi.u)^2/(2 cs4) - u.u/(2 cs2)],
    S = (1 - 1/(2 tau)) w [(xi - u)/cs2 + (xi.u) xi/cs4] . F,
    f(x + xi, t+1) = f - (f - feq)/tau + S."""
    d, c, w = oracle.lattice(lat)
    cs2 = 1.0 / 3.0
    nx, ny, nz = (list(dims) + [1, 1])[:3]
    rho = f.sum(1)
    F = np.asarray(fext, float)[:3]
    u = (f @ c.astype(float) + 0.5 * F[None, :]) / rho[:, None]
    cu = u @ c.T.astype(float)
    uu = (u * u).sum(1)
    feq = w[None, :] * rho[:, None] * (1 + cu / cs2 + cu ** 2 / (2 * cs2 ** 2)
                                       - uu[:, None] / (2 * cs2))
    xi_minus_u = c[None, :, :].astype(float) - u[:, None, :]
    S = (1 - 0.5 / tau) * w[None, :] * (
        (xi_minus_u @ F) / cs2 + cu * (c.astype(float) @ F)[None, :] / cs2 ** 2)
    post = f - (f - feq) / tau + S
    out = np.empty_like(f)
    grid = post.reshape(nz, ny, nx, -1)
    o = out.reshape(nz, ny, nx, -1)
    for i, (cx, cy, cz) in enumerate(c):
        o[..., i] = np.roll(grid[..., i], shift=(cz, cy, cx), axis=(0, 1, 2))
    return out


def _state(lat, dims, seed, eps=None):
    rng = np.random.default_rng(seed)
    n = oracle.ncells(dims)
    if eps is None:
        eps = rng.uniform(0.4, 1.0, n)
    u0 = rng.uniform(-0.05, 0.05, (_d(lat), n))
    f = oracle.init(lat, dims, eps, rng.uniform(0.9, 1.1, n), u0)
    return eps, f * rng.uniform(0.98, 1.02, f.shape)


@pytest.mark.parametrize("lat,dims", [(oracle.D2Q9, (6, 5)), (oracle.D3Q19, (4, 5, 3)),
                                      (oracle.D3Q27, (3, 4, 5))])
def test_bgk_step_matches_textbook_form(lat, dims):
    _, f = _state(lat, dims, 3, eps=np.ones(oracle.ncells(dims)))
    fext = [2e-4, -1e-4, 3e-4] if _d(lat) == 3 else [2e-4, -1e-4, 0.0]
    got = oracle.bgk_step(lat, dims, 0.7, f, fext)
    want = _textbook_bgk_guo(lat, dims, 0.7, f, fext)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-17)


@pytest.mark.parametrize("lat,dims", [(oracle.D2Q9, (8, 7)), (oracle.D3Q19, (5, 4, 6)),
                                      (oracle.D3Q27, (4, 4, 3)), (oracle.D2Q9, (1, 1)),
                                      (oracle.D3Q19, (1, 3, 2))])
def test_eps_one_reduces_to_bgk_bit_for_bit(lat, dims):
    n = oracle.ncells(dims)
    _, f = _state(lat, dims, 4, eps=np.ones(n))
    fext = [1e-6, 2e-6, -1e-6] if _d(lat) == 3 else [1e-6, 2e-6, 0.0]
    fa, fb = f.copy(), f.copy()
    for _ in range(25):
        fa = oracle.step(lat, dims, 0.8, np.ones(n), fa, fext=fext)
        fb = oracle.bgk_step(lat, dims, 0.8, fb, fext)
    assert np.array_equal(fa, fb)


@pytest.mark.parametrize("lat,dims", [(oracle.D2Q9, (8, 7)), (oracle.D3Q19, (5, 4, 6))])
def test_constant_eps_homogeneity(lat, dims):
    """phi == 1/2 with F/2 and f/2 gives exactly f/2 and the same rho, p, u."""
    n = oracle.ncells(dims)
    _, f = _state(lat, dims, 6, eps=np.ones(n))
    F = np.array([4e-5, -2e-5, 1e-5])
    fa, fb = f.copy(), 0.5 * f
    for _ in range(10):
        fa = oracle.step(lat, dims, 0.6, np.ones(n), fa, fext=F)
        fb = oracle.step(lat, dims, 0.6, np.full(n, 0.5), fb, fext=0.5 * F)
    assert np.array_equal(fb, 0.5 * fa)
    ra, pa, ua = oracle.moments(lat, dims, np.ones(n), fa, fext=F)
    rb, pb, ub = oracle.moments(lat, dims, np.full(n, 0.5), fb, fext=0.5 * F)
    assert np.array_equal(ra, rb) and np.array_equal(pa, pb) and np.array_equal(ua, ub)


@pytest.mark.parametrize("lat,dims", [(oracle.D2Q9, (16, 12)), (oracle.D3Q19, (8, 6, 5)),
                                      (oracle.D3Q27, (5, 6, 4))])
def test_mass_conserved_and_momentum_gains_force(lat, dims):
    rng = np.random.default_rng(7)
    n = oracle.ncells(dims)
    pert = rng.uniform(-0.2, 0.2, n)
    _, f = _state(lat, dims, 8, eps=0.75 + pert)
    fext = np.array([1e-5, -3e-6, 2e-6])
    m0, P0, _ = oracle.diagnostics(lat, dims, oracle.eps_at(dims, 0.75, pert, 40.0, 0), f,
                                   fext=fext)
    P_prev = P0
    for k in range(60):
        eps = oracle.eps_at(dims, 0.75, pert, 40.0, k)
        _, Pk, Fk = oracle.diagnostics(lat, dims, eps, f, fext=fext)
        f = oracle.step(lat, dims, 0.65, eps, f, fext=fext)
        eps1 = oracle.eps_at(dims, 0.75, pert, 40.0, k + 1)
        m1, P1, _ = oracle.diagnostics(lat, dims, eps1, f, fext=fext)
        assert abs(m1 - m0) <= 1e-13 * abs(m0)
        np.testing.assert_allclose(P1 - Pk, Fk, rtol=0, atol=1e-13 * abs(m0))


@pytest.mark.parametrize("lat,dims,shift", [(oracle.D2Q9, (7, 6), (2, 5, 0)),
                                            (oracle.D3Q19, (5, 4, 3), (1, 3, 2))])
def test_translation_covariance(lat, dims, shift):
    nx, ny, nz = (list(dims) + [1])[:3]
    eps, f = _state(lat, dims, 9)

    def roll_cells(a):
        g = a.reshape((nz, ny, nx) + a.shape[1:])
        return np.roll(g, shift=(shift[2], shift[1], shift[0]), axis=(0, 1, 2)).reshape(a.shape)

    out = oracle.step(lat, dims, 0.9, eps, f, fext=[1e-5, 0, 0])
    out_s = oracle.step(lat, dims, 0.9, roll_cells(eps), roll_cells(f), fext=[1e-5, 0, 0])
    assert np.array_equal(out_s, roll_cells(out))


@pytest.mark.parametrize("tau", [0.6, 0.9])
def test_shear_wave_viscosity(tau):
    """A shear wave u_x = A sin(k y) decays at rate nu k^2 with
    nu = (tau - 1/2)/3 (appendix, recovered viscosity); phi == 0.7 const."""
    N = 64
    dims = (4, N)
    n = oracle.ncells(dims)
    y = np.repeat(np.arange(N), 4)
    k = 2 * np.pi / N
    A = 1e-4
    eps = np.full(n, 0.7)
    u0 = np.vstack([A * np.sin(k * y), np.zeros(n)])
    f = oracle.init(oracle.D2Q9, dims, eps, None, u0)
    steps = 400
    amps = []
    for s in range(steps + 1):
        if s in (100, steps):
            _, _, u = oracle.moments(oracle.D2Q9, dims, eps, f)
            amps.append(2 * np.mean(u[0] * np.sin(k * y)))
        if s < steps:
            f = oracle.step(oracle.D2Q9, dims, tau, eps, f)
    nu = np.log(amps[0] / amps[1]) / ((steps - 100) * k * k)
    assert abs(nu / ((tau - 0.5) / 3.0) - 1.0) < 2e-3
