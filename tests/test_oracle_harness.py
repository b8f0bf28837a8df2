"""Pins of the oracle's initial state, time modulation and the plumbing of its
manufactured-solution harness.

  * initial state (eq. equilibrium): per cell, the populations' zeroth, first
    and second moments are rho0*phi, rho0*phi*u0 and rho0*phi*(u0 u0 + I/3);
  * time modulation of the separable volume fraction: m(0) = 1, m(T/2) = -1,
    m(T/4) = 0, the cosine recurrence m(n+1) + m(n-1) = 2 m(1) m(n), period
    and mirror symmetry; phi = eps_mean +/- pert at those levels;
  * the harness (phi(t_n) and F_MMS(t_n) per step, unit conversions, initial
    state, mean-free pressure and Euclidean velocity norms) against an
    independent loop written here: numpy fields from the sympy expressions of
    the printed examples, the VANSE residual derived symbolically, and
    ``oracle.step`` as the only shared piece.
"""
import numpy as np
import pytest
import sympy as sp

import oracle
from mms_fields import _momentum_residual, _paper_fields, t, x, y, z

LATS = [oracle.D2Q9, oracle.D3Q19, oracle.D3Q27]


@pytest.mark.parametrize("lat,dims", [(oracle.D2Q9, (7, 5)), (oracle.D3Q19, (5, 4, 3)),
                                      (oracle.D3Q27, (3, 5, 2))])
def test_init_moments_are_rho0_phi_and_u0(lat, dims):
    d, c, _ = oracle.lattice(lat)
    cc = c[:, :d].astype(float)
    n = oracle.ncells(dims)
    rng = np.random.default_rng(40 + lat)
    phi = rng.uniform(0.3, 1.0, n)
    rho0 = rng.uniform(0.8, 1.2, n)
    u0 = rng.uniform(-0.08, 0.08, (d, n))
    f = oracle.init(lat, dims, phi, rho0, u0)
    M0 = rho0 * phi
    np.testing.assert_allclose(f.sum(1), M0, rtol=1e-14)
    np.testing.assert_allclose(f @ cc, (M0 * u0).T, rtol=1e-12, atol=1e-16)
    second = np.einsum("ia,ib,ni->nab", cc, cc, f)
    want = M0[:, None, None] * (np.einsum("an,bn->nab", u0, u0) + np.eye(d)[None] / 3.0)
    np.testing.assert_allclose(second, want, rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("lat", LATS)
def test_init_defaults_are_unit_density_at_rest(lat):
    d, c, w = oracle.lattice(lat)
    dims = (4, 3) if d == 2 else (3, 2, 2)
    phi = np.linspace(0.5, 1.0, oracle.ncells(dims))
    f = oracle.init(lat, dims, phi)
    # at rest the equilibrium is w_i M0: the weights of Tables 1-2 times phi
    np.testing.assert_allclose(f, phi[:, None] * w[None, :], rtol=1e-15)


def test_modulation_special_values_and_recurrence():
    T = 1000.0
    assert oracle.modulation(0, T) == 1.0
    assert oracle.modulation(500, T) == -1.0
    assert abs(oracle.modulation(250, T)) < 1e-15
    assert abs(oracle.modulation(750, T)) < 1e-15
    for bad in (0.0, -5.0):
        assert oracle.modulation(123, bad) == 1.0  # no period: a static field
    m = np.array([oracle.modulation(n, T) for n in range(0, 2 * int(T) + 2)])
    # cos((n+1)a) + cos((n-1)a) = 2 cos(a) cos(n a)
    np.testing.assert_allclose(m[2:] + m[:-2], 2.0 * m[1] * m[1:-1], rtol=0, atol=1e-14)
    np.testing.assert_allclose(m[1000:2001], m[0:1001], rtol=0, atol=1e-14)   # period T
    np.testing.assert_allclose(m[1:500], m[999:500:-1], rtol=0, atol=1e-14)   # m(T-n) = m(n)
    assert np.all(np.abs(m) <= 1.0)
    # non-integer periods (the 2000-step period of the 64^2 workload, and T = 37.5)
    assert oracle.modulation(1000, 2000.0) == -1.0
    assert abs(oracle.modulation(75, 37.5) - 1.0) < 1e-15


def test_eps_at_is_mean_plus_modulated_perturbation():
    dims = (5, 4, 3)
    n = oracle.ncells(dims)
    pert = np.random.default_rng(3).uniform(-0.2, 0.2, n)
    np.testing.assert_array_equal(oracle.eps_at(dims, 0.7, pert, 40.0, 0), 0.7 + pert)
    np.testing.assert_array_equal(oracle.eps_at(dims, 0.7, pert, 40.0, 20), 0.7 - pert)
    np.testing.assert_allclose(oracle.eps_at(dims, 0.7, pert, 40.0, 10), np.full(n, 0.7),
                               rtol=0, atol=1e-16)
    np.testing.assert_array_equal(oracle.eps_at(dims, 0.7, None, 40.0, 13), np.full(n, 0.7))
    np.testing.assert_array_equal(oracle.eps_at(dims, 0.7, pert, 0.0, 13), 0.7 + pert)


def test_run_separable_equals_stepping_with_eps_at():
    """The driver loop: phi at t_n for step n, returned phi at the final level."""
    lat, dims = oracle.D3Q19, (4, 3, 5)
    n = oracle.ncells(dims)
    rng = np.random.default_rng(5)
    pert = rng.uniform(-0.15, 0.15, n)
    f0 = oracle.init(lat, dims, 0.75 + pert, None, rng.uniform(-0.02, 0.02, (3, n)))
    got, eps_end = oracle.run_separable(lat, dims, 0.7, 0.75, pert, 9.0, f0, 3, 7,
                                        fext=[1e-5, 0, 0])
    f = f0
    for k in range(3, 10):
        f = oracle.step(lat, dims, 0.7, 0.75 + np.cos(2 * np.pi * k / 9.0) * pert, f,
                        fext=[1e-5, 0, 0])
    np.testing.assert_allclose(got, f, rtol=1e-15, atol=1e-17)
    np.testing.assert_allclose(eps_end, 0.75 + np.cos(2 * np.pi * 10 / 9.0) * pert,
                               rtol=1e-15)


# ----------------------------------------------------------------------------
# Independent manufactured-solution loop
# ----------------------------------------------------------------------------
_LAMBDAS = {}


def _lambdas(ex):
    if ex not in _LAMBDAS:
        phi, u, p = _paper_fields(ex)
        F = _momentum_residual(phi, u, p)
        lam = lambda e: sp.lambdify((x, y, z, t), e, "numpy")  # noqa: E731
        _LAMBDAS[ex] = (lam(phi), [lam(e) for e in u], lam(p), [lam(e) for e in F])
    return _LAMBDAS[ex]


def _independent_mms(ex, N, tau, nsteps, time_offset=0):
    """Errors [u L1, L2, Linf, p L1, L2, Linf] after nsteps, in physical units,
    from a loop written from the validation section: L = 2 m periodic box,
    nodes at k*dx, nu = 0.1, rho = 1, diffusive scaling (dt = nu_lu dx^2/nu,
    nu_lu = (tau - 1/2)/3), velocity u dt/dx, pressure 1/3 + p (dt/dx)^2,
    force F dt^2/dx.  time_offset shifts the time level of phi and F (a
    planted mistake for the negative control)."""
    fphi, fu, fp, fF = _lambdas(ex)
    d = 3 if ex in (2, 5) else 2
    dims = (N, 1 if ex == 3 else N, N if d == 3 else 1)
    lat = oracle.D2Q9 if d == 2 else oracle.D3Q19
    quad = {1: 3, 2: 7, 3: 1, 4: 3, 5: 7}[ex]
    dx = 2.0 / N
    zz, yy, xx = np.meshgrid(np.arange(dims[2]) * dx, np.arange(dims[1]) * dx,
                             np.arange(dims[0]) * dx, indexing="ij")
    P = (xx.ravel(), yy.ravel(), zz.ravel())

    def ev(fn, tt):
        return np.broadcast_to(np.asarray(fn(*P, tt), dtype=float), P[0].shape).copy()

    dt = (tau - 0.5) / 3.0 * dx * dx / 0.1
    us, ps, fs = dt / dx, (dt / dx) ** 2, dt * dt / dx
    f = oracle.init(lat, dims, ev(fphi, 0.0), 3.0 * (1.0 / 3.0 + ev(fp, 0.0) * ps),
                    np.stack([ev(fu[a], 0.0) * us for a in range(d)]))
    for n in range(nsteps + 1):
        tn = (n + time_offset) * dt
        phi = ev(fphi, tn)
        force = np.stack([ev(fF[a], tn) * fs for a in range(3)])
        if n == nsteps:
            break
        f = oracle.step(lat, dims, tau, phi, f, quad_axes=quad, force=force, nthreads=1)
    _, p, u = oracle.moments(lat, dims, phi, f, quad_axes=quad, force=force)
    tn = nsteps * dt
    ue = np.stack([ev(fu[a], tn) for a in range(d)])
    pe = ev(fp, tn)
    du = np.sqrt(((u / us - ue) ** 2).sum(0))
    dp = np.abs((p - p.mean()) / ps - (pe - pe.mean()))
    return np.array([du.mean(), np.sqrt((du * du).mean()), du.max(),
                     dp.mean(), np.sqrt((dp * dp).mean()), dp.max()]), nsteps * dt


@pytest.mark.parametrize("ex", [1, 2, 3, 4, 5])
def test_mms_harness_matches_independent_loop(ex):
    tau = 0.53 if ex in (1, 2) else 0.5075
    want, t_end = _independent_mms(ex, 8, tau, 20)
    errs, _, n = oracle.mms_run(ex, 8, tau, t_end, n_samples=1, nthreads=1)
    assert n == 20
    # the stationary examples take F_MMS from central differences (h = 1e-4) in
    # the harness and from the exact residual here
    tol = 1e-7 if ex in (1, 2) else 1e-12
    np.testing.assert_allclose(errs[0], want, rtol=tol)


@pytest.mark.parametrize("ex", [3, 4, 5])
def test_mms_independent_loop_detects_a_time_level_shift(ex):
    """Negative control: phi and F one step late change the errors by far more
    than the tolerance above."""
    want, _ = _independent_mms(ex, 8, 0.5075, 20)
    late, _ = _independent_mms(ex, 8, 0.5075, 20, time_offset=1)
    assert np.max(np.abs(late - want) / want) > 1e-3
