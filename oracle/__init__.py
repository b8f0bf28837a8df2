"""CPU oracle of the consistent VANSE lattice Boltzmann step (arXiv:2208.09267).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2208_09267_amd``) never imports, links or calls it, and this package
imports nothing from the product path.

The arithmetic lives in plain C (``vanse_oracle.c``: the step, initial state,
moments and diagnostics; ``vanse_mms.c``: the manufactured-solution harness of
the paper's numerical validation), compiled in FP64 with ``-O2
-ffp-contract=off`` and no fast-math.  This module only marshals numpy arrays.

Layouts used here:
  * populations: AoS ``f[ncells, Q]`` with cells x-fastest,
    ``cell = (z*ny + y)*nx + x``;
  * scalar fields: ``[ncells]``; vector fields: SoA ``[d, ncells]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["vanse_oracle.c", "vanse_mms.c"]
_lock = threading.Lock()
_lib = None

D2Q9, D3Q19, D3Q27 = 0, 1, 2
QUAD_NONE = 8  # quad_axes value: no cell-integral correction (I = phi), ablation only
_Q = {D2Q9: 9, D3Q19: 19, D3Q27: 27}
_D = {D2Q9: 2, D3Q19: 3, D3Q27: 3}


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (plain gcc, FP64)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64P = ctypes.POINTER(ctypes.c_int64)
        i, d, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
        sig = {
            "oracle_lattice": (i, [i, P, P, P, P]),
            "oracle_quad_weights": (i, [i, P, P]),
            "oracle_step": (i, [i, I64P, d, P, i, P, P, P, P, i]),
            "oracle_bgk_step": (i, [i, I64P, d, P, P, P, i]),
            "oracle_feq": (i, [i, d, P, P]),
            "oracle_forcing": (i, [i, d, P, P, P]),
            "oracle_init": (i, [i, I64P, P, P, P, P]),
            "oracle_moments": (i, [i, I64P, P, i, P, P, P, P, P, P]),
            "oracle_diagnostics": (i, [i, I64P, P, i, P, P, P, P]),
            "oracle_modulation": (d, [i64, d]),
            "oracle_eps_at": (i, [I64P, d, P, d, i64, P]),
            "oracle_run_separable": (i, [i, I64P, d, d, P, d, i, P, P, i64, i64, P, P, P, i]),
            "oracle_mms_info": (i, [i, P, P, P]),
            "oracle_mms_fields_at": (i, [i, P, d, P, P, P]),
            "oracle_mms_force_fd": (i, [i, P, d, d, d, P]),
            "oracle_mms_force_exact": (i, [i, P, d, d, P]),
            "oracle_mms_run": (i64, [i, i, i, d, d, i, i, P, P]),
            "oracle_mms_run_q": (i64, [i, i, i, d, d, i, i, i, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims):
    d = list(dims) + [1] * (3 - len(dims))
    return (ctypes.c_int64 * 3)(*[int(v) for v in d])


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError("%s failed with status %d" % (what, rc))


def lattice(lat: int):
    """(d, xi[Q,3] int, w[Q]) of the oracle's own lattice tables."""
    lib = _load()
    d, q = ctypes.c_int(), ctypes.c_int()
    c = np.zeros((27, 3), dtype=np.int32)
    w = np.zeros(27)
    _check(lib.oracle_lattice(lat, ctypes.byref(d), ctypes.byref(q), _ptr(c), _ptr(w)),
           "oracle_lattice")
    return d.value, c[: q.value].astype(np.int64), w[: q.value].copy()


def quad_weights(n_axes: int):
    lib = _load()
    w0, wi = ctypes.c_double(), ctypes.c_double()
    _check(lib.oracle_quad_weights(n_axes, ctypes.byref(w0), ctypes.byref(wi)),
           "oracle_quad_weights")
    return w0.value, wi.value


def ncells(dims):
    d = list(dims) + [1] * (3 - len(dims))
    return int(d[0] * d[1] * d[2])


def step(lat, dims, tau, eps, f, quad_axes=0, force=None, fext=None, nthreads=0):
    """One time step; returns the new AoS populations."""
    lib = _load()
    eps, f, force = _f64(eps), _f64(f), _f64(force)
    fx = None if fext is None else _f64(list(fext) + [0.0] * (3 - len(fext)))
    out = np.empty_like(f)
    _check(lib.oracle_step(lat, _dims(dims), float(tau), _ptr(eps), int(quad_axes),
                           _ptr(force), _ptr(fx), _ptr(f), _ptr(out), int(nthreads)),
           "oracle_step")
    return out


def bgk_step(lat, dims, tau, f, fext=None, nthreads=0):
    lib = _load()
    f = _f64(f)
    fx = None if fext is None else _f64(list(fext) + [0.0] * (3 - len(fext)))
    out = np.empty_like(f)
    _check(lib.oracle_bgk_step(lat, _dims(dims), float(tau), _ptr(fx), _ptr(f), _ptr(out),
                               int(nthreads)), "oracle_bgk_step")
    return out


def feq(lat, M0, u):
    lib = _load()
    out = np.zeros(_Q[lat])
    uu = _f64(list(u) + [0.0] * (3 - len(u)))
    _check(lib.oracle_feq(lat, float(M0), _ptr(uu), _ptr(out)), "oracle_feq")
    return out


def forcing(lat, tau, u, F):
    lib = _load()
    out = np.zeros(_Q[lat])
    uu = _f64(list(u) + [0.0] * (3 - len(u)))
    FF = _f64(list(F) + [0.0] * (3 - len(F)))
    _check(lib.oracle_forcing(lat, float(tau), _ptr(uu), _ptr(FF), _ptr(out)),
           "oracle_forcing")
    return out


def init(lat, dims, eps0, rho0=None, u0=None):
    lib = _load()
    n = ncells(dims)
    eps0, rho0, u0 = _f64(eps0), _f64(rho0), _f64(u0)
    f = np.empty((n, _Q[lat]))
    _check(lib.oracle_init(lat, _dims(dims), _ptr(eps0), _ptr(rho0), _ptr(u0), _ptr(f)),
           "oracle_init")
    return f


def moments(lat, dims, eps, f, quad_axes=0, force=None, fext=None):
    """(rho, p, u[d, ncells]) at the time level of f and eps."""
    lib = _load()
    n = ncells(dims)
    eps, f, force = _f64(eps), _f64(f), _f64(force)
    fx = None if fext is None else _f64(list(fext) + [0.0] * (3 - len(fext)))
    rho, p, u = np.empty(n), np.empty(n), np.empty((_D[lat], n))
    _check(lib.oracle_moments(lat, _dims(dims), _ptr(eps), int(quad_axes), _ptr(force),
                              _ptr(fx), _ptr(f), _ptr(rho), _ptr(p), _ptr(u)),
           "oracle_moments")
    return rho, p, u


def diagnostics(lat, dims, eps, f, quad_axes=0, force=None, fext=None):
    """(mass, momentum[3], force_sum[3]) with compensated serial sums."""
    lib = _load()
    eps, f, force = _f64(eps), _f64(f), _f64(force)
    fx = None if fext is None else _f64(list(fext) + [0.0] * (3 - len(fext)))
    out = np.zeros(7)
    _check(lib.oracle_diagnostics(lat, _dims(dims), _ptr(eps), int(quad_axes), _ptr(force),
                                  _ptr(fx), _ptr(f), _ptr(out)), "oracle_diagnostics")
    return out[0], out[1:4].copy(), out[4:7].copy()


def modulation(n: int, period: float) -> float:
    return _load().oracle_modulation(int(n), float(period))


def eps_at(dims, eps_mean, pert, period, n):
    lib = _load()
    pert = _f64(pert)
    out = np.empty(ncells(dims))
    _check(lib.oracle_eps_at(_dims(dims), float(eps_mean), _ptr(pert), float(period),
                             int(n), _ptr(out)), "oracle_eps_at")
    return out


def run_separable(lat, dims, tau, eps_mean, pert, period, f, n0, nsteps, quad_axes=0,
                  force=None, fext=None, nthreads=0):
    """Advance f (AoS, modified copy returned) from step n0 by nsteps with
    phi(x, t_n) = eps_mean + cos(2 pi n / period) pert(x).  Returns
    (f, eps at t_{n0+nsteps})."""
    lib = _load()
    f = np.array(f, dtype=np.float64, copy=True, order="C")
    pert, force = _f64(pert), _f64(force)
    fx = None if fext is None else _f64(list(fext) + [0.0] * (3 - len(fext)))
    work = np.empty_like(f)
    eps_buf = np.empty(ncells(dims))
    _check(lib.oracle_run_separable(lat, _dims(dims), float(tau), float(eps_mean), _ptr(pert),
                                    float(period), int(quad_axes), _ptr(force), _ptr(fx),
                                    int(n0), int(nsteps), _ptr(f), _ptr(work), _ptr(eps_buf),
                                    int(nthreads)), "oracle_run_separable")
    return f, eps_buf


def mms_info(example: int):
    lib = _load()
    d, q, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib.oracle_mms_info(example, ctypes.byref(d), ctypes.byref(q), ctypes.byref(t)),
           "oracle_mms_info")
    return d.value, q.value, bool(t.value)


def mms_fields_at(example, X, t):
    lib = _load()
    XX = _f64(list(X) + [0.0] * (3 - len(X)))
    phi, p = ctypes.c_double(), ctypes.c_double()
    u = np.zeros(3)
    _check(lib.oracle_mms_fields_at(example, _ptr(XX), float(t), ctypes.byref(phi), _ptr(u),
                                    ctypes.byref(p)), "oracle_mms_fields_at")
    return phi.value, u, p.value


def mms_force_fd(example, X, t, nu=0.1, h=1e-4):
    lib = _load()
    XX = _f64(list(X) + [0.0] * (3 - len(X)))
    F = np.zeros(3)
    _check(lib.oracle_mms_force_fd(example, _ptr(XX), float(t), float(nu), float(h), _ptr(F)),
           "oracle_mms_force_fd")
    return F


def mms_force_exact(example, X, t, nu=0.1):
    lib = _load()
    XX = _f64(list(X) + [0.0] * (3 - len(X)))
    F = np.zeros(3)
    _check(lib.oracle_mms_force_exact(example, _ptr(XX), float(t), float(nu), _ptr(F)),
           "oracle_mms_force_exact")
    return F


def mms_run(example, N, tau, t_end, lat=None, n_samples=1, nthreads=0, quad_axes=None):
    """Run one manufactured-solution example at resolution N.  Returns
    (errors[n_samples, 6], times[n_samples], nsteps); the error columns are
    u L1, u L2, u Linf, p L1, p L2, p Linf in physical units.  quad_axes
    overrides the example's quadrature (QUAD_NONE: the ablation)."""
    lib = _load()
    d, _, _ = mms_info(example)
    if lat is None:
        lat = D2Q9 if d == 2 else D3Q19
    errs = np.zeros((n_samples, 6))
    times = np.zeros(n_samples)
    n = lib.oracle_mms_run_q(int(example), int(lat), int(N), float(tau), float(t_end),
                             int(n_samples), int(nthreads),
                             -1 if quad_axes is None else int(quad_axes), _ptr(errs),
                             _ptr(times))
    if n < 0:
        raise ValueError("oracle_mms_run failed with status %d" % n)
    return errs, times, int(n)
