"""GPU test of the handle's stream (vanse_set_stream, vanse_batch_set_stream):
the binding enqueues every call on torch's current stream, so a solve run
inside `torch.cuda.stream(side)` must produce exactly what it produces on the
default stream.  Covers the calls that synchronise on the handle's stream
(the 16-bit modes' init reduction, diagnostics), the two-step launch and a
graph-captured batch, for FP64, FP32 shifted and FP16; and two solves whose
launches interleave on two streams end where each ends alone.
"""
import numpy as np
import pytest
import torch

from paper_2208_09267_amd import vanse
from paper_2208_09267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(dtype, pert, u0, dims):
    s = vanse.Solver("D3Q19", dims, 0.6, dtype)
    s.set_porosity(0.75, pert, 20.0)
    s.set_force((1e-6, -2e-6, 5e-7))
    s.init(None, u0)
    s.step(3)                       # single steps, odd level
    s.set_fused(2, 4)
    s.step(7)                       # one single step to an even level, then two-step launches
    s.set_fused(0, 0)
    t = s.populations().cpu().numpy()
    mass, mom, fsum = s.diagnostics()
    d = [mass] + list(mom) + list(fsum)
    # a batch of this solve and a second one (graph-captured chunks of 4)
    s2 = vanse.Solver("D3Q19", dims, 0.8, dtype)
    s2.set_porosity(0.7, pert, 11.0)
    s2.init(None, u0)
    b = vanse.Batch([s, s2])
    b.set_tuning(256, 0, 4)
    b.step(10)
    b.close()
    out = (t, np.asarray(d), s.populations().cpu().numpy(), s2.populations().cpu().numpy())
    s.close()
    s2.close()
    return out


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FP32_SHIFTED, vanse.FP16_SHIFTED])
def test_side_stream_results_equal_the_default_stream(dtype):
    dims = (64, 12, 10)
    pert = torch.from_numpy(W.fourier_eps(dims, seed=7)).cuda()
    u0 = torch.from_numpy(np.ascontiguousarray(W.taylor_green(dims, 0.03))).cuda()
    ref = _run(dtype, pert, u0, dims)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got = _run(dtype, pert, u0, dims)
    torch.cuda.current_stream().wait_stream(side)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_two_solves_interleaved_on_two_streams_equal_sequential_runs():
    """Handles share no device state: two solves whose launches are enqueued
    alternately on two streams (so they may overlap on the device) end
    bitwise where each ends alone."""
    dims = (64, 16, 12)
    pert = torch.from_numpy(W.fourier_eps(dims, seed=9)).cuda()
    u0 = torch.from_numpy(np.ascontiguousarray(W.taylor_green(dims, 0.02))).cuda()

    def make(tau, dtype, fused):
        s = vanse.Solver("D3Q19", dims, tau, dtype)
        s.set_porosity(0.75, pert, 13.0)
        s.init(None, u0)
        if fused:
            s.set_fused(4, 4)
        return s

    cases = [(0.6, vanse.FP32_SHIFTED, True), (0.9, vanse.FP16_SHIFTED, False)]
    alone = []
    for c in cases:
        s = make(*c)
        s.step(24)
        alone.append(s.populations().cpu().numpy())
        s.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    solvers = []
    for c, st in zip(cases, streams):
        with torch.cuda.stream(st):
            solvers.append(make(*c))
    for _ in range(12):
        for s, st in zip(solvers, streams):
            with torch.cuda.stream(st):
                s.step(2)
    for s, st, ref in zip(solvers, streams, alone):
        with torch.cuda.stream(st):
            got = s.populations().cpu().numpy()
        assert np.array_equal(got, ref)
    for st in streams:
        torch.cuda.current_stream().wait_stream(st)
    for s in solvers:
        s.close()
