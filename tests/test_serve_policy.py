"""CPU tests of the serving loop's host logic: the admission policy (a pure
function of the budget and the queue), how far the batch runs between host
visits, and the state-size formula."""
import pytest

from paper_2208_09267_amd import serve, vanse

GB = 1 << 30


def test_fcfs_admits_while_budget_and_cells_allow():
    qb, qc = [10 * GB, 20 * GB, 5 * GB], [100, 200, 50]
    assert serve.admit_count(qb, qc, 0, 0, 0, 100 * GB, 10_000, 64) == 3
    assert serve.admit_count(qb, qc, 75 * GB, 0, 0, 100 * GB, 10_000, 64) == 1
    # the head blocks: the small third request does not overtake the second
    assert serve.admit_count(qb, qc, 75 * GB, 0, 1, 100 * GB, 10_000, 64) == 1
    assert serve.admit_count(qb, qc, 95 * GB, 0, 1, 100 * GB, 10_000, 64) == 0


def test_cell_cap_and_member_cap():
    qb, qc = [1, 1, 1, 1], [40, 40, 40, 40]
    assert serve.admit_count(qb, qc, 0, 0, 0, 100, 100, 64) == 2
    assert serve.admit_count(qb, qc, 0, 30, 1, 100, 100, 64) == 1
    assert serve.admit_count(qb, qc, 0, 0, 0, 100, 1000, 3) == 3
    assert serve.admit_count(qb, qc, 0, 0, 62, 100, 1000, 64) == 2


def test_idle_gpu_admits_one_oversized_request_but_never_over_budget():
    assert serve.admit_count([5], [10_000], 0, 0, 0, 10, 100, 64) == 1
    assert serve.admit_count([5, 5], [10_000, 1], 0, 0, 0, 10, 100, 64) == 1
    assert serve.admit_count([50], [1], 0, 0, 0, 10, 100, 64) == 0
    assert serve.admit_count([], [], 0, 0, 0, 10, 100, 64) == 0


def test_steps_until_host():
    # nothing queued, requests still to arrive: stop at the chunk boundary
    assert serve.steps_until_host(500, 16, False, True) == 16
    assert serve.steps_until_host(7, 16, False, True) == 7
    # the queue head waits for memory: nothing joins before the next retirement
    assert serve.steps_until_host(500, 16, True, True) == 500
    # no request left to arrive: run to the next retirement
    assert serve.steps_until_host(500, 16, False, False) == 500
    assert serve.steps_until_host(3, 16, True, False) == 3


@pytest.mark.parametrize("dtype,elem,pert", [(vanse.FP64, 8, 8), (vanse.FP32_SHIFTED, 4, 4),
                                             (vanse.FP16_SHIFTED, 2, 4),
                                             (vanse.FX16_SHIFTED, 2, 4)])
def test_state_bytes_formula(dtype, elem, pert):
    n = 33 * 17 * 5
    stride = (n + 127) // 128 * 128
    want = 19 * stride * elem + stride * pert + 8 * (7 * 1024 + 64)
    assert serve.state_bytes("D3Q19", (33, 17, 5), dtype) == want
    # the two-step launch's second population array
    assert serve.state_bytes("D3Q19", (33, 17, 5), dtype, two_step=True) == want + 19 * stride * elem
    assert serve.state_bytes("D2Q9", (33, 17, 1), dtype, two_step=True) == \
        serve.state_bytes("D2Q9", (33, 17, 1), dtype)


def _autotune_steps(t, odd_start):
    """Real steps vanse_batch_autotune takes with t steps per trial: six
    single-step trials, one aligning step when the members sit at an odd
    level, then twice a two-step trial (t rounded up to a multiple of 4) and
    twice the best single-step candidate (t rounded up to even)."""
    return 6 * t + (1 if (odd_start + 6 * t) % 2 else 0) + 2 * ((t + 3) // 4 * 4) + 2 * ((t + 1) // 2 * 2)


def test_tune_trial_steps_stay_within_every_member():
    assert serve.tune_trial_steps(10_000) == 16
    assert serve.tune_trial_steps(18) == 0
    assert serve.tune_trial_steps(19) == 1
    assert serve.tune_trial_steps(500, longest=4) == 4
    for m in range(0, 400):
        t = serve.tune_trial_steps(m)
        assert 0 <= t <= 16
        if t:
            assert max(_autotune_steps(t, o) for o in (0, 1)) <= m
    # the 2-step trial of the GPU autotune test: 12 + 2 * (4 + 2)
    assert _autotune_steps(2, 0) == 24


def test_retune_rule():
    assert serve.retune(0, 16) and serve.retune(0, 3)   # no choice yet, a trial fits
    assert not serve.retune(0, 0)                       # nothing fits
    assert not serve.retune(16, 16)                     # a full-length choice stays
    assert not serve.retune(3, 8)                       # still short: keep the choice
    assert serve.retune(3, 16)                          # short choice, full trial fits now
