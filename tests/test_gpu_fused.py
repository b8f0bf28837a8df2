"""GPU tests of the two-step launch (temporal blocking, vanse_set_fused).

One launch advances two time levels through an LDS tile that marches in z.
It must be bitwise equal to two single steps for every tile shape, storage
mode and 3-D lattice: from even and odd time levels, with odd step counts,
ragged z-segments, one-tile lattices (the tile's outer rows are its own
rows), a per-cell force field and periodic wrap in every direction.  It is
also checked against the CPU oracle directly, for its argument checks, and
for batches whose members switched arrays while stepping alone.
"""
import zlib

import numpy as np
import pytest
import torch

from gpu_helpers import direction_map, oracle_run, rel_linf
from paper_2208_09267_amd import vanse
from paper_2208_09267_amd import workloads as W

pytestmark = pytest.mark.gpu


def _compiled(lat, dtype, dims, rows):
    """Mirror of the shape rule in vanse_set_fused's documentation."""
    nx, ny = dims[0], dims[1]
    i = -(-nx * rows // 512)
    h = -(-nx * (rows + 2) // 512)
    if rows > ny:
        return False
    if nx % 64 == 0 and ny % rows == 0:
        if lat == "D3Q27":
            return dtype != vanse.FP64 and (h <= 3 if i == 1 else
                                            (i == 2 and (h == 2 or (nx == 256 and rows == 4))))
        if dtype == vanse.FP64:
            return i == 1 and h <= 2
        return i <= 2 and h <= i + 2
    if lat == "D3Q27":
        return dtype != vanse.FP64 and i == 1 and h <= 2
    if dtype == vanse.FP64:
        return i == 1 and h == 1
    return h <= 3 if i == 1 else (i == 2 and h == 2)


def _solver(lat, dims, dtype, seed, force_field=False):
    n = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    s = vanse.Solver(lat, dims, float(rng.uniform(0.52, 1.0)), dtype)
    s.set_porosity(0.75, torch.from_numpy(W.fourier_eps(dims, seed=seed)).cuda(),
                   float(rng.uniform(9, 40)))
    s.set_force((1e-6, -2e-6, 3e-7))
    if force_field:
        s.set_force_field(torch.from_numpy(rng.uniform(-1e-4, 1e-4, (3, n))).cuda())
    s.init(torch.from_numpy(rng.uniform(0.98, 1.02, n)).cuda(),
           torch.from_numpy(np.ascontiguousarray(W.taylor_green(dims, 0.03))).cuda())
    return s


def _state(s):
    f = s.populations().cpu().numpy()
    rho, p, u = (t.cpu().numpy() for t in s.moments())
    return f, rho, p, u


def _pair(lat, dims, dtype, rows, planes, pre, steps, seed, force_field=False):
    """(single-step state, two-step state) after pre + steps steps; the
    two-step launch is switched on after `pre` single steps."""
    out = []
    for fused in (False, True):
        s = _solver(lat, dims, dtype, seed, force_field)
        s.step(pre)
        if fused:
            s.set_fused(rows, planes)
        s.step(steps)
        assert s.time == pre + steps
        out.append(_state(s))
        s.close()
    return out


SHAPES = [("D3Q19", (64, 8, 6), 1, 4), ("D3Q19", (64, 8, 6), 2, 32), ("D3Q19", (64, 8, 6), 4, 1),
          ("D3Q19", (64, 8, 6), 8, 3), ("D3Q19", (128, 4, 5), 2, 2), ("D3Q19", (64, 2, 1), 2, 8),
          ("D3Q19", (64, 1, 2), 1, 1), ("D3Q19", (192, 6, 7), 3, 5), ("D3Q19", (256, 4, 9), 4, 4),
          ("D3Q19", (128, 12, 3), 6, 2),
          # the compile-time tiles of the benchmarked launches: 128 x 4 (the
          # 128^3 workload, 16-plane segments) and 256 x 2 (FP64 at 256^3,
          # 128-plane segments, here with a 2-plane last segment)
          ("D3Q19", (128, 8, 20), 4, 16), ("D3Q19", (256, 4, 130), 2, 128),
          ("D3Q27", (64, 4, 5), 2, 2), ("D3Q27", (64, 8, 6), 8, 4), ("D3Q27", (128, 6, 4), 3, 3),
          ("D3Q27", (64, 3, 1), 3, 1), ("D3Q27", (256, 4, 5), 4, 3), ("D3Q27", (256, 8, 3), 4, 2),
          # general tiles: nx not a multiple of 64, rows not dividing ny (shorter last tile)
          ("D3Q19", (48, 10, 7), 4, 3), ("D3Q19", (33, 17, 5), 5, 2), ("D3Q19", (96, 7, 6), 3, 4),
          ("D3Q19", (7, 5, 3), 2, 1), ("D3Q19", (1, 1, 1), 1, 1), ("D3Q19", (64, 9, 4), 4, 8),
          ("D3Q19", (130, 3, 2), 2, 2), ("D3Q27", (40, 6, 5), 4, 3), ("D3Q27", (17, 3, 2), 2, 1)]


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FP32_SHIFTED, vanse.FP16_SHIFTED,
                                   vanse.FX16_SHIFTED])
@pytest.mark.parametrize("lat,dims,rows,planes", SHAPES)
def test_two_step_equals_single_steps_bitwise(lat, dims, rows, planes, dtype):
    print("case", lat, dims, rows, planes, dtype, flush=True)
    if not _compiled(lat, dtype, dims, rows):
        s = _solver(lat, dims, dtype, 1)
        with pytest.raises(vanse.VanseError) as e:
            s.set_fused(rows, planes)
        assert e.value.code == vanse.EINVAL
        s.close()
        return
    seed = zlib.crc32(repr((lat, dims, rows, planes)).encode()) % 1000
    for pre, steps in ((0, 9), (1, 10), (3, 3)):
        (f1, *m1), (f2, *m2) = _pair(lat, dims, dtype, rows, planes, pre, steps, seed,
                                     force_field=(pre == 1))
        assert np.array_equal(f1, f2), (pre, steps)
        for a, b in zip(m1, m2):
            assert np.array_equal(a, b), (pre, steps)


def test_two_step_vs_oracle_every_population():
    dims, steps = (64, 4, 5), 12
    rng = np.random.default_rng(5)
    n = int(np.prod(dims))
    pert, u0, rho0 = rng.uniform(-0.2, 0.2, n), rng.uniform(-0.04, 0.04, (3, n)), \
        rng.uniform(0.97, 1.03, n)
    s = vanse.Solver("D3Q19", dims, 0.58, vanse.FP64)
    s.set_porosity(0.7, torch.from_numpy(pert).cuda(), 11.0)
    s.set_force((2e-5, -1e-5, 3e-5))
    s.init(torch.from_numpy(rho0).cuda(), torch.from_numpy(u0).cuda())
    s.set_fused(2, 2)
    s.step(steps)
    f_gpu, rho, p, u = _state(s)
    s.close()
    f_o, rho_o, p_o, u_o = oracle_run("D3Q19", dims, 0.58, 0.7, pert, 11.0, steps, u0=u0,
                                      rho0=rho0, force=(2e-5, -1e-5, 3e-5))
    perm = direction_map("D3Q19")
    for k in range(f_o.shape[1]):
        assert rel_linf(f_gpu[perm[k]], f_o[:, k]) <= 1e-12, k
    for a, b in ((rho, rho_o), (p, p_o), (u, u_o)):
        assert rel_linf(a, b) <= 1e-12


def test_set_fused_argument_checks_and_memory():
    s = _solver("D3Q19", (64, 6, 4), vanse.FP32_SHIFTED, 2)
    base = s.device_bytes
    for rows, planes in ((7, 1), (1, 0), (-1, 4), (16, 4)):  # 7 > ny, planes 0, negative, 16 rows
        with pytest.raises(vanse.VanseError) as e:
            s.set_fused(rows, planes)
        assert e.value.code == vanse.EINVAL
    s.set_fused(3, 2)
    pop = 19 * 4 * ((64 * 6 * 4 + 127) // 128 * 128)
    assert s.device_bytes == base + pop
    s.step(4)
    s.set_fused(0)
    assert s.device_bytes == base
    s.step(3)
    assert s.time == 7
    s.close()
    for lat, dims in (("D3Q19", (600, 4, 4)), ("D2Q9", (64, 4, 1))):  # no shape, 2-D
        s = vanse.Solver(lat, dims, 0.7, vanse.FP32_SHIFTED)
        with pytest.raises(vanse.VanseError) as e:
            s.set_fused(2, 2)
        assert e.value.code == vanse.EINVAL
        s.close()


def test_batch_after_two_step_solo_steps_matches_single_steps():
    dtype = vanse.FP32_SHIFTED
    cases = [((64, 8, 6), 1), ((128, 4, 5), 2), ((64, 6, 7), 3)]
    ref = []
    for dims, seed in cases:
        s = _solver("D3Q19", dims, dtype, seed)
        s.step(6 + 11 + 4)
        ref.append(s.populations().cpu().numpy())
        s.close()
    mem = [_solver("D3Q19", dims, dtype, seed) for dims, seed in cases]
    b = vanse.Batch(mem)
    b.step(6)
    for m in mem:  # alone, two-step: each member ends on its second array
        m.set_fused(2, 3)
        m.step(11)
    b.step(4)      # the batch must follow the members to their current arrays
    for m, r in zip(mem, ref):
        assert m.time == 21
        assert np.array_equal(m.populations().cpu().numpy(), r)
    b.close()
    for m in mem:
        m.close()

