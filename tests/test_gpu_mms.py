"""The travelling manufactured solutions (Examples 3-5 of the numerical
validation) on the GPU, in FP64 through the C ABI.

Every step the volume fraction phi(t_n) and the manufactured force
F_MMS(t_n) change; both are generated on the device by a test-only input
kernel (tests/mms_input_kernel.hip, checked here against the torch statement
tests/mms_inputs.py, which is pinned against the symbolic residual on the CPU)
and handed to the solver as a full phi field (vanse_set_porosity with
eps_mean 0 and no modulation) and a per-cell force field, with the quadrature
of each example (D1Q3 along x for Example 3, D2Q5, D3Q7).

  * parity: the same inputs drive the CPU oracle's step; every population
    agrees to 1e-11 relative after a few hundred steps;
  * second order: velocity and mean-free pressure errors (physical units,
    Euclidean norm per node, L1/L2/Linf) converge at ~2 in every norm on
    Example 4 from N = 36 to 48 and Example 5 from N = 24 to 32 (tau =
    0.5075, diffusive scaling), errors taken once stabilised (at 12 s and
    40 s).
"""
import numpy as np
import pytest
import torch

import mms_device
import mms_inputs as MI
import oracle
from gpu_helpers import direction_map
from paper_2208_09267_amd import vanse

pytestmark = pytest.mark.gpu
ORACLE_LAT = {"D2Q9": oracle.D2Q9, "D3Q19": oracle.D3Q19}


def gpu_mms(ex, N, tau, nsteps, samples=(), populations=False, progress=False):
    """Run Example ex at N on the GPU for nsteps steps.  Returns the errors
    [u L1, L2, Linf, p L1, L2, Linf] at each step count in `samples` (and at
    nsteps), and optionally the final populations.  progress: print a line
    at every sample."""
    lat, dims, d, quad, dx, dt, us, ps, fs = MI.setup(ex, N, tau)
    dev = torch.device("cuda")
    phi, u, p, F = MI.fields(ex, N, 0.0, dev)
    s = vanse.Solver(lat, dims, tau, vanse.FP64)
    s.set_porosity(0.0, phi, 0.0, quad)
    s.init(1.0 + 3.0 * p * ps, (u[:d] * us).contiguous())
    errs = {}
    want = sorted(set(list(samples) + [nsteps]))
    n_cells = phi.numel()
    phi_t = torch.empty(n_cells, dtype=torch.float64, device=dev)
    force_t = torch.empty(d, n_cells, dtype=torch.float64, device=dev)
    for n in range(nsteps + 1):
        mms_device.travel_fields(ex, N, n * dt, fs, phi_t, force_t)
        s.set_porosity(0.0, phi_t, 0.0, quad)
        s.set_force_field(force_t)
        if n in want:
            _, u, p, _ = MI.fields(ex, N, n * dt, dev)
            _, pl, ul = s.moments()
            du = ((ul / us - u[:d]) ** 2).sum(0).sqrt()
            dp = ((pl - pl.mean()) / ps - (p - p.mean())).abs()
            errs[n] = np.array([float(du.mean()), float((du * du).mean().sqrt()), float(du.max()),
                                float(dp.mean()), float((dp * dp).mean().sqrt()), float(dp.max())])
            if progress:
                print("example %d N %d step %d/%d errors %s" % (ex, N, n, nsteps, errs[n]),
                      flush=True)
        elif progress and n % 100000 == 0:
            print("example %d N %d step %d/%d" % (ex, N, n, nsteps), flush=True)
        if n == nsteps:
            break
        s.step(1)
    f = s.populations().cpu().numpy() if populations else None
    s.close()
    return errs, f


def oracle_mms(ex, N, tau, nsteps):
    """The oracle's step driven by the same inputs: the input kernel's arrays
    copied to the host (the force padded with a zero z plane in 2-D)."""
    lat, dims, d, quad, dx, dt, us, ps, fs = MI.setup(ex, N, tau)
    L = ORACLE_LAT[lat]
    phi, u, p, F = MI.fields(ex, N, 0.0, "cuda")
    f = oracle.init(L, dims, phi.cpu().numpy(), (1.0 + 3.0 * p * ps).cpu().numpy(),
                    (u[:d] * us).cpu().numpy())
    n_cells = phi.numel()
    phi_t = torch.empty(n_cells, dtype=torch.float64, device="cuda")
    force_t = torch.empty(d, n_cells, dtype=torch.float64, device="cuda")
    force3 = np.zeros((3, n_cells))
    for n in range(nsteps):
        mms_device.travel_fields(ex, N, n * dt, fs, phi_t, force_t)
        force3[:d] = force_t.cpu().numpy()
        f = oracle.step(L, dims, tau, phi_t.cpu().numpy(), f, quad_axes=quad, force=force3)
    return f


@pytest.mark.parametrize("ex,N", [(3, 40), (4, 24), (5, 12)])
def test_input_kernel_matches_the_torch_fields(ex, N):
    lat, dims, d, quad, dx, dt, us, ps, fs = MI.setup(ex, N, 0.5075)
    n = int(np.prod(dims))
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    force = torch.empty(d, n, dtype=torch.float64, device="cuda")
    for t in (0.0, 0.731, 5.3):
        mms_device.travel_fields(ex, N, t, 1.0, phi, force)
        w_phi, _, _, w_F = MI.fields(ex, N, t, "cuda")
        torch.testing.assert_close(phi, w_phi, rtol=1e-14, atol=1e-15)
        torch.testing.assert_close(force, w_F[:d], rtol=1e-12, atol=1e-12 * float(w_F.abs().max()))


@pytest.mark.parametrize("ex,N,steps", [(3, 16, 400), (4, 16, 300), (5, 10, 200)])
def test_travelling_examples_every_population_vs_oracle(ex, N, steps):
    print("case", ex, N, steps, flush=True)
    lat = MI.setup(ex, N, 0.5075)[0]
    _, f_gpu = gpu_mms(ex, N, 0.5075, steps, populations=True)
    f_o = oracle_mms(ex, N, 0.5075, steps)
    perm = direction_map(lat)
    for k in range(f_o.shape[1]):
        a, b = f_gpu[perm[k]], f_o[:, k]
        assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max(), k


# The travelling fields repeat every 4 s (sin(pi (x - t/2))), and so do the
# error norms once the state has stabilised: errors are compared at the same
# phase, t_end - 4 s and t_end.  Example 4 has stabilised by 8 s; Example 5's
# velocity error keeps growing towards its stabilised value with a time
# constant of about 8 s (u L1 +27% from 8 s to 40 s at N = 16), so it runs to
# 40 s.
PERIOD_S = 4.0


def _stable_errors(ex, N, tau, t_end):
    dt = MI.setup(ex, N, tau)[5]
    nsteps = int(round(t_end / dt))
    samples = [nsteps - int(round(PERIOD_S / dt)), nsteps]
    errs, _ = gpu_mms(ex, N, tau, nsteps, samples=samples, progress=True)
    last, prev = errs[samples[-1]], errs[samples[-2]]
    assert np.all(np.abs(last - prev) <= 0.05 * last), (N, errs)
    return last


@pytest.mark.parametrize("ex,Ns,t_end", [(4, (36, 48), 12.0), (5, (24, 32), 40.0)])
def test_travelling_examples_second_order_on_gpu(ex, Ns, t_end):
    print("case", ex, Ns, flush=True)
    e = [_stable_errors(ex, N, 0.5075, t_end) for N in Ns]
    order = np.log(e[0] / e[1]) / np.log(Ns[1] / Ns[0])
    print("errors", e, "order", order, flush=True)
    assert np.all(order > 1.7) and np.all(order < 2.3), order
