"""GPU tests of the continuous-batching loop: every request's result is
bitwise identical when served alone and when served in a mix of requests
that arrive while others are on the GPU; a bad request fails alone."""
import numpy as np
import pytest

from paper_2208_09267_amd import serve, vanse
from paper_2208_09267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(77)
    out = []
    for r in range(9):
        n = int(rng.integers(12, 40))
        dims = (n, int(rng.integers(10, 30)), int(rng.integers(8, 24)))
        steps = int(rng.integers(30, 130))
        tau = float(rng.uniform(0.55, 1.0))
        out.append((0.004 * r, W.Workload("t%d" % r, "D3Q19", dims, tau, steps, 0.75, 100.0,
                                          seed=500 + r, tgv_amp=0.02)))
    return out


@pytest.mark.parametrize("autotune", [True, False])
@pytest.mark.parametrize("dtype", [vanse.FP32_SHIFTED, vanse.FP64])
def test_results_identical_alone_and_in_mix(dtype, autotune):
    # mix: autotuned, or the two-step batched launch (requests joining at the
    # batch's parity); alone: single steps only
    reqs = _requests()
    mixed = serve.Server(dtype=dtype, keep_fields=True, chunk=16, autotune=autotune).run(reqs)
    assert all(r.error is None for r in mixed)
    for (ta, w), got in zip(reqs, mixed):
        alone = serve.Server(dtype=dtype, keep_fields=True, chunk=16, autotune=False,
                             two_step=False).run([(0.0, w)])[0]
        assert alone.error is None
        assert np.array_equal(alone.rho, got.rho), w.name
        assert np.array_equal(alone.p, got.p), w.name
        assert np.array_equal(alone.u, got.u), w.name


def test_requests_overlap_on_the_device():
    reqs = [(0.0, W.Workload("long", "D3Q19", (48, 48, 48), 0.6, 400, 0.75, 100.0, seed=1,
                             tgv_amp=0.02))]
    reqs += [(0.002 * k, W.Workload("s%d" % k, "D3Q19", (16, 16, 16), 0.7, 40, 0.75, 100.0,
                                    seed=2 + k, tgv_amp=0.02)) for k in range(1, 6)]
    srv = serve.Server(chunk=8, autotune=False)
    res = srv.run(reqs)
    long_ = res[0]
    # short requests were admitted and finished while the long one was in flight
    assert all(r.admit < long_.finish and r.finish < long_.finish for r in res[1:])
    assert srv.stats["rebuilds"] >= 2


def test_bad_request_fails_alone():
    reqs = _requests()[:4]
    bad = W.Workload("bad", "D3Q19", (10, 10, 10), 0.5, 20, 0.75, 100.0, seed=9)
    mix = reqs[:2] + [(0.001, bad)] + reqs[2:]
    res = serve.Server(keep_fields=True).run(mix)
    assert res[2].error is not None and "tau" in res[2].error
    good = [r for r in res if r.error is None]
    assert len(good) == 4
    for (ta, w), got in zip(reqs, good):
        alone = serve.Server(keep_fields=True, autotune=False, two_step=False).run([(0.0, w)])[0]
        assert np.array_equal(alone.u, got.u)


def test_over_budget_request_is_refused():
    big = W.Workload("big", "D3Q19", (64, 64, 64), 0.7, 10, 0.75, 100.0, seed=3)
    small = W.Workload("small", "D3Q19", (8, 8, 8), 0.7, 10, 0.75, 100.0, seed=4)
    budget = serve.state_bytes("D3Q19", (32, 32, 32), vanse.FP32_SHIFTED)
    res = serve.Server(budget_bytes=budget).run([(0.0, big), (0.0, small)])
    assert res[0].error is not None and "budget" in res[0].error
    assert res[1].error is None


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FP32_SHIFTED, vanse.FP16_SHIFTED,
                                   vanse.FX16_SHIFTED])
def test_state_bytes_matches_library(dtype):
    for dims in [(8, 8, 8), (33, 17, 5), (1, 1, 1)]:
        s = vanse.Solver("D3Q19", dims, 0.7, dtype)
        assert s.device_bytes == serve.state_bytes("D3Q19", dims, dtype)
        s.set_fused(1, 4)  # the second population array of the two-step launch
        assert s.device_bytes == serve.state_bytes("D3Q19", dims, dtype, two_step=True)
        s.close()
