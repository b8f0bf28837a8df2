"""The manufactured solutions of the paper's numerical validation (Examples
1-5, rho = 1) as sympy expressions, the VANSE residuals, and numpy
evaluators on a lattice, shared by the oracle tests and the GPU
convergence tests.  Written from the printed formulas; Example 5 in the
travelling reading (the printed form violates the mass equation)."""
import numpy as np
import sympy as sp

x, y, z, t = sp.symbols("x y z t", real=True)
X = (x, y, z)
pi = sp.pi


def _paper_fields(ex, corrected=True):
    """Fields as printed in the numerical-validation section (rho = 1)."""
    s = sp.sin
    c = sp.cos
    if ex == 1:
        phi = sp.Rational(1, 2) + sp.Rational(2, 5) * s(pi * x) * s(pi * y)
        u = (2 * (-(s(pi * x) ** 2) * s(pi * y) * c(pi * y)),
             2 * (s(pi * y) ** 2) * s(pi * x) * c(pi * x), 0)
        p = s(pi * x) * s(pi * y)
    elif ex == 2:
        phi = sp.Rational(1, 2) + sp.Rational(2, 5) * s(pi * x) * s(pi * y) * s(pi * z)
        u = (s(pi * x) ** 2 * s(pi * y) * c(pi * y) * s(pi * z) * c(pi * z),
             s(pi * y) ** 2 * s(pi * x) * c(pi * x) * s(pi * z) * c(pi * z),
             -2 * s(pi * z) ** 2 * s(pi * x) * c(pi * x) * s(pi * y) * c(pi * y))
        p = s(pi * x) * s(pi * y) * s(pi * z)
    elif ex == 3:
        phi = sp.Rational(1, 2) + sp.Rational(2, 5) * s(pi * (x - t / 2))
        u = (sp.Rational(1, 2) + 1 / phi, 0, 0)
        p = s(pi * (x - t / 2))
    elif ex == 4:
        arg = s(pi * (x - t / 2)) * s(pi * (y - t / 2))
        phi = sp.Rational(1, 2) + sp.Rational(2, 5) * arg
        u = (sp.Rational(1, 2) + 1 / phi, sp.Rational(1, 2) + 1 / phi, 0)
        p = arg
    elif ex == 5:
        if corrected:
            arg = s(pi * (x - t / 2)) * s(pi * (y - t / 2)) * s(pi * (z - t / 2))
        else:
            arg = s(pi * x) * s(pi * y) * s(pi * z)
        phi = sp.Rational(1, 2) + sp.Rational(2, 5) * arg
        u = tuple(sp.Rational(1, 2) + 1 / phi for _ in range(3))
        p = arg
    return phi, u, p


def _mass_residual(phi, u):
    return sp.diff(phi, t) + sum(sp.diff(phi * u[a], X[a]) for a in range(3))


def _momentum_residual(phi, u, p, nu=sp.Rational(1, 10)):
    F = []
    for a in range(3):
        term = sp.diff(phi * u[a], t) + phi * sp.diff(p, X[a])
        for b in range(3):
            term += sp.diff(phi * u[a] * u[b], X[b])
            term -= nu * sp.diff(phi * (sp.diff(u[a], X[b]) + sp.diff(u[b], X[a])), X[b])
        F.append(term)
    return F


def mms_arrays(ex, N, time, nu=0.1, L=2.0):
    """phi, u[3], p and F_MMS[3] (physical units) at the nodes x_k = k L/N of
    the example's lattice (N x N, N x 1 for Example 3, N^3 in 3-D), flattened
    x fastest."""
    phi, u, p = _paper_fields(ex)
    F = _momentum_residual(phi, u, p, nu=sp.Rational(str(nu)))
    dim = 3 if ex in (2, 5) else 2
    dims = (N, 1 if ex == 3 else N, N if dim == 3 else 1)
    dx = L / N
    zz, yy, xx = np.meshgrid(np.arange(dims[2]) * dx, np.arange(dims[1]) * dx,
                             np.arange(dims[0]) * dx, indexing="ij")
    args = (xx.ravel(), yy.ravel(), zz.ravel(), float(time))
    ev = lambda e: np.broadcast_to(np.asarray(sp.lambdify((x, y, z, t), e, "numpy")(*args),
                                              dtype=float), xx.size).copy()
    return dims, ev(phi), np.stack([ev(e) for e in u]), ev(p), np.stack([ev(e) for e in F])
