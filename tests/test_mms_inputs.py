"""CPU pin of the torch input generator of the travelling manufactured
solutions (tests/mms_inputs.py) against the sympy expressions of the printed
examples and the symbolically derived VANSE momentum residual."""
import numpy as np
import pytest
import sympy as sp

import mms_inputs as MI
from mms_fields import _momentum_residual, _paper_fields, t, x, y, z


@pytest.mark.parametrize("ex,N", [(3, 16), (4, 12), (5, 6)])
@pytest.mark.parametrize("time", [0.0, 0.37, 3.1])
def test_torch_inputs_match_the_symbolic_fields_and_residual(ex, N, time):
    phi, u, p = _paper_fields(ex)
    F = _momentum_residual(phi, u, p)
    lam = lambda e: sp.lambdify((x, y, z, t), e, "numpy")  # noqa: E731
    dims = MI.setup(ex, N, 0.6)[1]
    dx = MI.L / N
    zz, yy, xx = np.meshgrid(np.arange(dims[2]) * dx, np.arange(dims[1]) * dx,
                             np.arange(dims[0]) * dx, indexing="ij")
    P = (xx.ravel(), yy.ravel(), zz.ravel(), time)
    ev = lambda e: np.broadcast_to(np.asarray(lam(e)(*P), dtype=float), xx.size)  # noqa: E731
    g_phi, g_u, g_p, g_F = (a.numpy() for a in MI.fields(ex, N, time))
    np.testing.assert_allclose(g_phi, ev(phi), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(g_p, ev(p), rtol=1e-13, atol=1e-14)
    for a in range(3):
        np.testing.assert_allclose(g_u[a], ev(u[a]), rtol=1e-13, atol=1e-14)
        want = ev(F[a])
        np.testing.assert_allclose(g_F[a], want, rtol=1e-11, atol=1e-11 * np.abs(want).max())


def test_setup_scalings_follow_diffusive_scaling():
    lat, dims, d, quad, dx, dt, us, ps, fs = MI.setup(4, 32, 0.5075)
    assert (lat, dims, d, quad) == ("D2Q9", (32, 32, 1), 2, 3)
    nu_lu = 0.0075 / 3.0
    assert dx == 2.0 / 32 and abs(dt - nu_lu * dx * dx / 0.1) < 1e-18
    assert abs(us - dt / dx) < 1e-18 and abs(ps - us * us) < 1e-20 and abs(fs - dt * dt / dx) < 1e-20
