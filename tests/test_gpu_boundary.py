"""GPU tests of the C ABI's error paths and parameter changes.

  * a rejected vanse_set_porosity / vanse_set_force_field (NaN, phi outside
    (0, 1]) leaves the solver exactly as it was: the run continues bitwise as
    if the call had not been made;
  * non-finite arithmetic (a finite force far beyond any physical value)
    makes vanse_diagnostics return EUNSTABLE, and every later vanse_step and
    batch step refuses (sticky); in the 16-bit fixed-point mode so does a
    state outside its range;
  * the 16-bit codes are relative to the mean initial M0 (a dense state
    stays in range), and vanse_init refuses a rho0 whose mean is not
    positive;
  * a member whose phi or force changes after the batch was built is stepped
    with the new parameters (bitwise equal to the same changes made alone).
"""
import numpy as np
import pytest
import torch

from paper_2208_09267_amd import vanse
from paper_2208_09267_amd import workloads as W

pytestmark = pytest.mark.gpu
DIMS = (24, 20, 18)


def _solver(dtype=vanse.FP64, dims=DIMS, seed=3, force_field=False, tau=0.7):
    n = int(np.prod(dims))
    s = vanse.Solver("D3Q19", dims, tau, dtype)
    s.set_porosity(0.75, torch.from_numpy(W.fourier_eps(dims, seed=seed)).cuda(), 30.0)
    s.set_force((1e-6, -2e-6, 5e-7))
    if force_field:
        rng = np.random.default_rng(seed)
        s.set_force_field(torch.from_numpy(rng.uniform(-1e-4, 1e-4, (3, n))).cuda())
    s.init(None, torch.from_numpy(np.ascontiguousarray(W.taylor_green(dims, 0.02))).cuda())
    return s


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FP32_SHIFTED])
def test_rejected_set_porosity_leaves_the_solver_unchanged(dtype):
    n = int(np.prod(DIMS))
    ref = _solver(dtype)
    ref.step(11)
    want = ref.populations().cpu().numpy()
    ref.close()

    s = _solver(dtype)
    s.step(5)
    nan = torch.from_numpy(W.fourier_eps(DIMS, seed=9)).cuda()
    nan[123] = float("nan")
    with pytest.raises(vanse.VanseError) as e:
        s.set_porosity(0.75, nan, 30.0)
    assert e.value.code == vanse.EINVAL
    big = torch.full((n,), 0.4, dtype=torch.float64, device="cuda")
    with pytest.raises(vanse.VanseError) as e:
        s.set_porosity(0.75, big, 30.0)          # phi would reach 1.15
    assert e.value.code == vanse.EINVAL
    with pytest.raises(vanse.VanseError) as e:
        s.set_porosity(0.0, None, 0.0)           # phi = 0
    assert e.value.code == vanse.EINVAL
    s.step(6)
    assert s.time == 11
    assert np.array_equal(s.populations().cpu().numpy(), want)
    s.close()


def test_rejected_force_field_leaves_the_solver_unchanged():
    n = int(np.prod(DIMS))
    ref = _solver(force_field=True)
    ref.step(9)
    want = ref.populations().cpu().numpy()
    ref.close()

    s = _solver(force_field=True)
    s.step(4)
    for bad in (float("nan"), float("inf"), -float("inf")):
        F = torch.zeros(3, n, dtype=torch.float64, device="cuda")
        F[1, 77] = bad
        with pytest.raises(vanse.VanseError) as e:
            s.set_force_field(F)
        assert e.value.code == vanse.EINVAL
    s.step(5)
    assert np.array_equal(s.populations().cpu().numpy(), want)
    s.close()
    # a first call that is rejected allocates nothing and switches nothing on
    t = _solver()
    before = t.device_bytes
    F = torch.full((3, n), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(vanse.VanseError):
        t.set_force_field(F)
    assert t.device_bytes == before
    t.close()


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FX16_SHIFTED])
@pytest.mark.parametrize("fused", [False, True])
def test_non_finite_arithmetic_makes_the_solver_unstable(fused, dtype):
    """FX16 stores no NaN: the overflowing values saturate at the bound of
    its range, which reads back as NaN."""
    s = _solver(dtype)
    if fused:
        s.set_fused(1, 4)
    s.step(4)
    m, _, _ = s.diagnostics()
    assert np.isfinite(m)
    # finite, so accepted; the velocity it drives overflows u.u to infinity
    s.set_force((1e300, 0.0, 0.0))
    s.step(2)
    with pytest.raises(vanse.VanseError) as e:
        s.diagnostics()
    assert e.value.code == vanse.EUNSTABLE
    with pytest.raises(vanse.VanseError) as e:
        s.step(1)
    assert e.value.code == vanse.EUNSTABLE
    assert s.time == 6
    with pytest.raises(vanse.VanseError) as e:   # sticky
        s.diagnostics()
    assert e.value.code == vanse.EUNSTABLE
    # a batch refuses a member that is unstable
    ok = _solver(dtype, seed=4)
    b = vanse.Batch([ok, s])
    with pytest.raises(vanse.VanseError) as e:
        b.step(2)
    assert e.value.code == vanse.EUNSTABLE
    b.close()
    # re-initialising clears the state
    s.set_force((0.0, 0.0, 0.0))
    s.init()
    s.step(2)
    assert np.isfinite(s.diagnostics()[0])
    ok.close()
    s.close()


def _rho0(value, dims=DIMS):
    return torch.full((int(np.prod(dims)),), value, dtype=torch.float64, device="cuda")


def test_fx16_unit_keeps_a_dense_state_in_range():
    """rho0 = 2 with phi in [0.5, 1] on a small grid (steep phi): M0 spans
    [1, 2] and the populations reach 2.8 w_i.  In units of the mean initial
    M0 (c ~ 1.5) the code h = f/(c w) - 1 stays within (-1, 1) over the run
    (checked on the FP64 populations); in units of 1 it would leave it and
    saturate.  The FX16 run stays finite and close to FP64 (2^-16 c w
    rounding per step)."""
    pert = torch.from_numpy(W.fourier_eps(DIMS, seed=3)).cuda()
    u0 = torch.from_numpy(np.ascontiguousarray(W.taylor_green(DIMS, 0.01))).cuda()
    c = float((2.0 * (0.75 + pert)).mean())
    w = np.array(vanse.lattice_info(vanse.D3Q19)[2])[:, None]
    out = []
    for dt in (vanse.FP64, vanse.FX16_SHIFTED):
        s = vanse.Solver("D3Q19", DIMS, 0.7, dt)
        s.set_porosity(0.75, pert, 30.0)
        s.init(_rho0(2.0), u0)
        f0 = s.populations().cpu().numpy()
        hmax = np.abs(f0 / (c * w) - 1.0).max()
        h1 = np.abs(f0 / w - 1.0).max()
        for _ in range(4):
            s.step(10)
            f = s.populations().cpu().numpy()
            hmax = max(hmax, np.abs(f / (c * w) - 1.0).max())
            h1 = max(h1, np.abs(f / w - 1.0).max())
        if dt == vanse.FP64:
            print("FP64 rho0 2: max |f/(c w) - 1|", hmax, "max |f/w - 1|", h1, flush=True)
            assert hmax < 0.95 and h1 > 1.0
        m = s.diagnostics()[0]
        out.append((f0, m, [t.cpu().numpy() for t in s.moments()]))
        s.close()
    (f64, m64, (r64, p64, u64)), (f16, m16, (r, p, u)) = out
    # initial populations: each within half a step of the code, c w 2^-16
    # (plus the FP32 rounding of f/(c w) - 1 before it is coded)
    assert np.all(np.abs(f16 - f64) <= c * w * (2.0 ** -16 + 1e-7))
    er, eu = np.abs(r - r64).max() / np.abs(r64).max(), np.abs(u - u64).max() / np.abs(u64).max()
    print("FX16 rho0 2: mass", (m16 - m64) / m64, "rho", er, "u", eu, flush=True)
    assert abs(m16 - m64) <= 1e-6 * m64
    assert er <= 1e-4 and eu <= 5e-4


def test_fx16_state_outside_its_range_is_unstable_and_init_validates_the_centre():
    n = int(np.prod(DIMS))
    s = _solver(vanse.FX16_SHIFTED)
    s.step(3)
    # a cell 5 times denser than the rest: f/(c w) - 1 ~ 4 there, beyond +-1
    rho0 = _rho0(1.0)
    rho0[777] = 5.0
    s.init(rho0)
    f = s.populations().cpu().numpy()
    assert np.all(np.isnan(f[:, 777])) and np.all(np.isfinite(np.delete(f, 777, axis=1)))
    with pytest.raises(vanse.VanseError) as e:
        s.diagnostics()
    assert e.value.code == vanse.EUNSTABLE
    with pytest.raises(vanse.VanseError) as e:
        s.step(1)
    assert e.value.code == vanse.EUNSTABLE
    s.init()
    s.step(2)
    assert np.isfinite(s.diagnostics()[0])
    # a rho0 whose mean is not finite and positive is refused before
    # anything changes: the run continues as if the call had not been made
    ref = _solver(vanse.FX16_SHIFTED)
    ref.step(7)
    want = ref.populations().cpu().numpy()
    ref.close()
    t = _solver(vanse.FX16_SHIFTED)
    t.step(3)
    for bad in (float("nan"), 0.0, -1.0):
        with pytest.raises(vanse.VanseError) as e:
            t.init(_rho0(bad))
        assert e.value.code == vanse.EINVAL
    assert t.time == 3
    t.step(4)
    assert np.array_equal(t.populations().cpu().numpy(), want)
    t.close()
    s.close()
    assert n > 777


@pytest.mark.parametrize("flags", [0, vanse.TUNE_TWO_STEP])
def test_batch_member_parameter_changes_take_effect(flags):
    dtype = vanse.FP32_SHIFTED
    specs = [((32, 32, 32), 0.8, 5), ((48, 40, 36), 0.62, 6)]
    new_pert = torch.from_numpy(W.fourier_eps((48, 40, 36), seed=99)).cuda()
    n0 = 32 * 32 * 32
    field = torch.from_numpy(np.random.default_rng(1).uniform(-1e-5, 1e-5, (3, n0))).cuda()

    def change(a, b):
        a.set_force((3e-6, 1e-6, -2e-6))
        a.set_force_field(field)
        b.set_porosity(0.7, new_pert, 25.0, 3)

    solo = [_solver(dtype, d, seed, tau=t) for d, t, seed in specs]
    for s in solo:
        s.step(8)
    change(*solo)
    for s in solo:
        s.step(12)
    want = [s.populations().cpu().numpy() for s in solo]

    mem = [_solver(dtype, d, seed, tau=t) for d, t, seed in specs]
    b = vanse.Batch(mem)
    b.set_tuning(256, flags, 16)
    b.step(8)
    change(*mem)
    b.step(12)
    for k, s in enumerate(mem):
        assert s.time == 20
        assert np.array_equal(s.populations().cpu().numpy(), want[k]), k
    b.close()
    for s in solo + mem:
        s.close()
