"""Write oracle reference values for the full-size GPU parity tests.

Calls only the CPU oracle (``oracle``) and the seeded input recipes
(``paper_2208_09267_amd.workloads``).  For each workload it runs the full
number of steps in FP64 and stores, in ``<name>.npz``:
  cells        sampled cell indices (fixed seed) plus the eight corners
  rho, p, u    the oracle's fields at those cells at the final time
  norms        L-infinity norms over ALL cells of rho, p, u and of p - mean(p)
  mass         sum over all cells of sum_i f_i (compensated)
  steps        number of steps run

Usage: python tests/golden/make_golden.py d3q19_128 [d3q19_256]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2208_09267_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NSAMPLES = 4096


def sample_cells(dims):
    nx, ny, nz = dims
    n = nx * ny * nz
    rng = np.random.default_rng(12345)
    picks = set(int(c) for c in rng.choice(n, size=min(NSAMPLES, n), replace=False))
    for z in (0, nz - 1):
        for y in (0, ny - 1):
            for x in (0, nx - 1):
                picks.add((z * ny + y) * nx + x)
    return np.array(sorted(picks), dtype=np.int64)


def run(name):
    w = getattr(W, name)()
    lat = oracle.D2Q9 if w.lattice == "D2Q9" else oracle.D3Q19
    pert = w.eps_pert()
    eps0 = oracle.eps_at(w.dims, w.eps_mean, pert, w.period, 0)
    f = oracle.init(lat, w.dims, eps0, None, w.u0())
    t0 = time.time()
    done = 0
    chunk = 50
    while done < w.steps:
        k = min(chunk, w.steps - done)
        f, eps = oracle.run_separable(lat, w.dims, w.tau, w.eps_mean, pert, w.period, f, done, k,
                                      quad_axes=w.quad_axes, fext=w.force)
        done += k
        print("%s: %d/%d steps, %.0f s" % (name, done, w.steps, time.time() - t0), flush=True)
    rho, p, u = oracle.moments(lat, w.dims, eps, f, quad_axes=w.quad_axes, fext=w.force)
    mass, _, _ = oracle.diagnostics(lat, w.dims, eps, f, quad_axes=w.quad_axes, fext=w.force)
    cells = sample_cells(w.dims)
    norms = np.array([np.abs(rho).max(), np.abs(p).max(), np.abs(u).max(),
                      np.abs(p - p.mean()).max()])
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, cells=cells, rho=rho[cells], p=p[cells], u=u[:, cells],
                        norms=norms, mass=np.array(mass), steps=np.array(w.steps))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["d3q19_128"]:
        run(name)
