"""GPU tests of the batched workload at its full size, in the launch the
benchmark times: the 64 solves (edges 32/48/64/96, tau in [0.55, 1], own
seeded phi each) advanced 500 steps by the autotuned batched launch (whose
trial steps are real steps).  FP32 shifted: a member of every size is
bitwise equal to the same solve stepped alone by the single-step kernel.
FP64: a member of each of the three smaller sizes matches the CPU oracle to
1e-11 relative L-infinity in rho, p and u."""
import numpy as np
import pytest
import torch

from gpu_helpers import oracle_run, rel_linf
from paper_2208_09267_amd import vanse
from paper_2208_09267_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 500


def _solver(w, dtype):
    s = vanse.Solver(w.lattice, w.dims, w.tau, dtype)
    s.set_porosity(w.eps_mean, torch.from_numpy(w.eps_pert()).cuda(), w.period)
    s.init(None, torch.from_numpy(np.ascontiguousarray(w.u0())).cuda())
    return s


def _run_batch(ws, dtype):
    solvers = [_solver(w, dtype) for w in ws]
    b = vanse.Batch(solvers)
    block, flags, run = b.autotune(5)
    print("batched launch", block, flags, run, flush=True)
    b.step(STEPS - run)
    b.close()
    assert all(s.time == STEPS for s in solvers)
    return solvers, flags


def _first_of_each_size(ws, sizes):
    out = {}
    for k, w in enumerate(ws):
        if w.dims[0] in sizes and w.dims[0] not in out:
            out[w.dims[0]] = k
    return [out[n] for n in sorted(out)]


def test_batched_64_fp32_members_equal_solo_bitwise():
    ws = W.batched_64()
    solvers, flags = _run_batch(ws, vanse.FP32_SHIFTED)
    assert flags & vanse.TUNE_TWO_STEP  # the launch the benchmark reports
    for k in _first_of_each_size(ws, (32, 48, 64, 96)):
        print("member", k, ws[k].dims, flush=True)
        solo = _solver(ws[k], vanse.FP32_SHIFTED)
        solo.step(STEPS)
        assert np.array_equal(solo.populations().cpu().numpy(),
                              solvers[k].populations().cpu().numpy()), k
        solo.close()
    for s in solvers:
        s.close()


def test_batched_64_fp64_members_vs_oracle():
    ws = W.batched_64()
    solvers, _ = _run_batch(ws, vanse.FP64)
    for k in _first_of_each_size(ws, (32, 48, 64)):
        w = ws[k]
        print("member", k, w.dims, flush=True)
        rho, p, u = (t.cpu().numpy() for t in solvers[k].moments())
        _, rho_o, p_o, u_o = oracle_run(w.lattice, w.dims, w.tau, w.eps_mean, w.eps_pert(),
                                        w.period, STEPS, u0=w.u0())
        errs = [rel_linf(a, b) for a, b in ((rho, rho_o), (p, p_o), (u, u_o))]
        print("rel Linf rho %.3e p %.3e u %.3e" % tuple(errs), flush=True)
        assert max(errs) <= 1e-11, errs
    for s in solvers:
        s.close()
