"""GPU tests of the batched launch: every solve in a batch evolves bitwise
identically to the same solve stepped alone (uneven sizes, different tau,
phi, force and time level / AA parity), across graph chunks, per-step
launches and every autotuned launch shape."""
import numpy as np
import pytest
import torch

from paper_2208_09267_amd import vanse
from paper_2208_09267_amd import workloads as W

pytestmark = pytest.mark.gpu

# small enough that the general tiles of the batched two-step launch take
# z-segments of at most 8 planes (the batch cannot fill the GPU with 32)
CASES = [((17, 13, 11), 0.57, 1), ((32, 32, 32), 0.9, 2), ((48, 40, 36), 0.66, 3),
         ((5, 64, 7), 0.75, 4), ((64, 8, 9), 1.2, 5)]


def _balanced(nz, target):
    """Planes per segment when nz is split into equal segments of at most
    `target` planes."""
    segs = -(-nz // target)
    return -(-nz // segs)


def _make(dims, tau, seed, dtype, pre_steps=0):
    pert = W.fourier_eps(dims, seed=seed)
    s = vanse.Solver("D3Q19", dims, tau, dtype)
    s.set_porosity(0.75, torch.from_numpy(pert).cuda(), 40.0 + seed)
    s.set_force((1e-6 * seed, -2e-7, 3e-7))
    s.init(None, torch.from_numpy(np.ascontiguousarray(W.taylor_green(dims, 0.02))).cuda())
    if pre_steps:
        s.step(pre_steps)
    return s


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FP32_SHIFTED, vanse.FP16_SHIFTED,
                                   vanse.FX16_SHIFTED])
@pytest.mark.parametrize("steps,chunk", [(37, 16), (5, 0), (32, 16)])
def test_batch_matches_solo_bitwise(dtype, steps, chunk):
    print("case", dtype, steps, chunk, flush=True)
    pre = [0, 3, 0, 1, 2]  # members start at different time levels (parities)
    solo = [_make(d, t, s, dtype, p) for (d, t, s), p in zip(CASES, pre)]
    for s in solo:
        s.step(steps)
    want = [s.populations().cpu().numpy() for s in solo]
    for s in solo:
        s.close()

    members = [_make(d, t, s, dtype, p) for (d, t, s), p in zip(CASES, pre)]
    b = vanse.Batch(members)
    b.set_tuning(256, 0, chunk)
    b.step(steps)
    for k, s in enumerate(members):
        assert s.time == pre[k] + steps
        got = s.populations().cpu().numpy()
        assert np.array_equal(got, want[k]), k
    b.close()
    for s in members:
        s.close()


def test_autotune_keeps_results_bitwise():
    dtype = vanse.FP32_SHIFTED
    solo = [_make(d, t, s, dtype) for d, t, s in CASES]
    members = [_make(d, t, s, dtype) for d, t, s in CASES]
    b = vanse.Batch(members)
    block, flags, run = b.autotune(2)
    assert block in (64, 128, 256) and flags in (0, 1, 16, 17)
    # 6 single-step trials of 2 steps, then twice a two-step trial of 4 and the
    # best single-step candidate on 2
    assert run in (0, 24)
    b.step(20)
    for s in solo:
        s.step(run + 20)
    for s, m in zip(solo, members):
        assert m.time == s.time
        assert np.array_equal(s.populations().cpu().numpy(), m.populations().cpu().numpy())
    b.close()
    # second batch of the same size class: the choice comes from the cache
    b2 = vanse.Batch(members)
    assert b2.autotune(2) == (block, flags, 0)
    assert b2.autotune(1) == (block, flags, 0)  # shorter trials: the cached choice
    assert b2.autotune(3)[2] >= 6 * 3           # longer trials run again
    assert b2.autotune(3)[2] == 0               # and replace it
    b2.close()
    for s in solo + members:
        s.close()


def test_batch_rejects_mixed_or_uninitialised_members():
    a = _make((8, 8, 8), 0.7, 1, vanse.FP64)
    c = _make((8, 8, 8), 0.7, 1, vanse.FP32_SHIFTED)
    with pytest.raises(vanse.VanseError) as e:
        vanse.Batch([a, c])
    assert e.value.code == vanse.EINVAL
    u = vanse.Solver("D3Q19", (8, 8, 8), 0.7)
    with pytest.raises(vanse.VanseError) as e:
        vanse.Batch([a, u])
    assert e.value.code == vanse.ESTATE
    with pytest.raises(vanse.VanseError):
        vanse.Batch([a, a])
    for s in (a, c, u):
        s.close()


def test_batch_update_changes_members_and_stays_bitwise():
    dtype = vanse.FP32_SHIFTED
    solo = [_make(d, t, s, dtype) for d, t, s in CASES]
    mem = [_make(d, t, s, dtype) for d, t, s in CASES]
    b = vanse.Batch(mem[:2])
    b.step(7)
    b.update(mem[1:5])          # drop one, add three (different time levels)
    b.step(20)
    b.update(mem)               # grow past the first capacity
    b.step(3)
    b.update([mem[4]])
    b.step(5)
    steps = [10, 30, 23, 23, 28]
    for s, n in zip(solo, steps):
        s.step(n)
    for s, m, n in zip(solo, mem, steps):
        assert m.time == n
        assert np.array_equal(s.populations().cpu().numpy(), m.populations().cpu().numpy())
    b.close()
    for s in solo + mem:
        s.close()


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FP32_SHIFTED, vanse.FP16_SHIFTED,
                                   vanse.FX16_SHIFTED])
@pytest.mark.parametrize("steps,chunk", [(37, 16), (10, 0), (32, 16)])
def test_two_step_batch_matches_solo_bitwise(dtype, steps, chunk):
    """Members at even levels advance by two-step launches (general tiles for
    every size; FP64 members wider than 170 cells keep single steps)."""
    print("case", dtype, steps, chunk, flush=True)
    pre = [0, 2, 0, 4, 2]
    solo = [_make(d, t, s, dtype, p) for (d, t, s), p in zip(CASES, pre)]
    for s in solo:
        s.step(steps)
    want = [s.populations().cpu().numpy() for s in solo]
    for s in solo:
        s.close()
    members = [_make(d, t, s, dtype, p) for (d, t, s), p in zip(CASES, pre)]
    b = vanse.Batch(members)
    b.set_tuning(128, vanse.TUNE_TWO_STEP, chunk)
    if dtype != vanse.FP64:
        # every member at most 96 wide: 768-thread general tiles (rows
        # 768/nx - 2, at most ny), in equal z-segments of one target
        lay = b.two_step_layout()
        assert [r for r, _ in lay] == [13, 22, 14, 64, 8]
        assert any(all(p == _balanced(d[2], t) for p, (d, _, _) in zip([p for _, p in lay], CASES))
                   for t in (32, 24, 16, 12, 8))
    b.step(steps)
    for k, s in enumerate(members):
        assert s.time == pre[k] + steps
        assert np.array_equal(s.populations().cpu().numpy(), want[k]), k
    # the batch keeps going after a member stepped alone (two-step, odd count)
    members[1].set_fused(1, 4)
    members[1].step(3)
    b.step(8)
    ref = _make(*CASES[1], dtype, pre[1])
    ref.step(steps + 3 + 8)
    assert np.array_equal(members[1].populations().cpu().numpy(), ref.populations().cpu().numpy())
    ref.close()
    b.close()
    for s in members:
        s.close()


def test_autotune_does_not_cache_an_untried_two_step_launch():
    dtype = vanse.FP16_SHIFTED  # D3Q27 in FP16: a tuning-cache key no other test uses
    pre = [0, 1, 0, 1, 0]
    members = [_make_lat("D3Q27", d, t, s, dtype, p) for (d, t, s), p in zip(CASES, pre)]
    b = vanse.Batch(members)
    block, flags, run = b.autotune(1)
    assert run == 6 and not flags & vanse.TUNE_TWO_STEP  # mixed parity: single steps only
    b.close()
    for m in members:
        if m.time % 2:
            m.step(1)
    b = vanse.Batch(members)
    block, flags, run = b.autotune(1)
    assert run == 6 + 2 * (4 + 2)  # not cached: the two-step candidate is tried now
    b.close()
    b = vanse.Batch(members)
    assert b.autotune(1) == (block, flags, 0)
    b.close()
    for m in members:
        m.close()


def test_two_step_batch_mixed_parity_falls_back_to_single_steps():
    dtype = vanse.FP32_SHIFTED
    pre = [0, 1, 2, 3, 0]
    solo = [_make(d, t, s, dtype, p) for (d, t, s), p in zip(CASES, pre)]
    members = [_make(d, t, s, dtype, p) for (d, t, s), p in zip(CASES, pre)]
    b = vanse.Batch(members)
    b.set_tuning(256, vanse.TUNE_TWO_STEP, 16)
    b.step(20)
    for s, m in zip(solo, members):
        s.step(20)
        assert np.array_equal(s.populations().cpu().numpy(), m.populations().cpu().numpy())
    b.close()
    for s in solo + members:
        s.close()


# Members that share a compile-time tile of the single-solve launch (every
# member as wide as the tile, its rows dividing ny) run the batched two-step
# kernel with that tile; any other mix uses general tiles.
TILE_GROUPS = {
    "256x4": [((256, 8, 6), 0.6, 11), ((256, 4, 9), 0.8, 12), ((256, 12, 3), 1.1, 13)],
    "256x2": [((256, 6, 5), 0.6, 14), ((256, 2, 3), 0.9, 15)],  # ny not a multiple of 4
    "128x4": [((128, 8, 5), 0.7, 16), ((128, 4, 7), 0.95, 17)],
    "mixed": [((256, 4, 4), 0.7, 18), ((128, 4, 5), 0.8, 19)],
}


def _make_lat(lat, dims, tau, seed, dtype, pre_steps=0):
    pert = W.fourier_eps(dims, seed=seed)
    s = vanse.Solver(lat, dims, tau, dtype)
    s.set_porosity(0.75, torch.from_numpy(pert).cuda(), 40.0 + seed)
    s.set_force((1e-6 * seed, -2e-7, 3e-7))
    s.init(None, torch.from_numpy(np.ascontiguousarray(W.taylor_green(dims, 0.02))).cuda())
    if pre_steps:
        s.step(pre_steps)
    return s


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FP32_SHIFTED, vanse.FP16_SHIFTED,
                                   vanse.FX16_SHIFTED])
@pytest.mark.parametrize("lat", ["D3Q19", "D3Q27"])
@pytest.mark.parametrize("group", list(TILE_GROUPS))
def test_two_step_batch_compile_time_tiles_bitwise(group, lat, dtype):
    print("case", group, lat, dtype, flush=True)
    cases = TILE_GROUPS[group]
    pre = [0, 2, 4][:len(cases)]
    steps = 37
    solo = [_make_lat(lat, d, t, s, dtype, p) for (d, t, s), p in zip(cases, pre)]
    for s in solo:
        s.step(steps)
    want = [s.populations().cpu().numpy() for s in solo]
    for s in solo:
        s.close()
    members = [_make_lat(lat, d, t, s, dtype, p) for (d, t, s), p in zip(cases, pre)]
    b = vanse.Batch(members)
    b.set_tuning(256, vanse.TUNE_TWO_STEP, 16)
    b.step(steps)
    for k, s in enumerate(members):
        assert s.time == pre[k] + steps
        assert np.array_equal(s.populations().cpu().numpy(), want[k]), k
    b.close()
    for s in members:
        s.close()


def _xt_tile(nx, ny, f64):
    """(columns, rows) of a member's tile in a batch with x-split members,
    whose kernel has one interior and one halo cell per thread (FP64) or two
    and two: full rows where they fit (FP64 up to 170 wide, reduced storage
    up to 341), else the fewest segments of at most 62 columns, one wave per
    row, and 6 (FP64) or 14 rows."""
    per = 1 if f64 else 2
    full = min(per * 512 // nx - 2, ny)
    if nx <= (170 if f64 else 341) or nx <= 62:
        return (nx, full) if full >= 1 else (0, 0)
    k = -(-nx // 62)
    return -(-nx // k), min(per * 8 - 2, ny)


@pytest.mark.parametrize("dtype", [vanse.FP32_SHIFTED, vanse.FP16_SHIFTED, vanse.FX16_SHIFTED])
def test_two_step_batch_24_plane_segments_bitwise(dtype):
    """Four requests of the served stream's sizes (edges 80, 63, 153, 69:
    4.7 M cells) have too few general tiles to fill the GPU with 32-plane
    z-segments; the batched launch splits their nz into equal segments of at
    most 24 planes (153: 7 of 22, 80: 4 of 20), and every member still
    equals the solve stepped alone."""
    print("case 24-plane segments", dtype, flush=True)
    cases = [((80, 80, 80), 0.6, 21), ((63, 63, 63), 0.85, 22), ((153, 153, 153), 0.7, 23),
             ((69, 69, 69), 0.95, 24)]
    steps = 21
    solo = [_make_lat("D3Q19", d, t, s, dtype) for d, t, s in cases]
    for s in solo:
        s.step(steps)
    want = [s.populations().cpu().numpy() for s in solo]
    for s in solo:
        s.close()
    members = [_make_lat("D3Q19", d, t, s, dtype) for d, t, s in cases]
    b = vanse.Batch(members)
    b.set_tuning(256, vanse.TUNE_TWO_STEP, 16)
    # rows: as many full x-rows as fit 512 interior and 1024 halo-plane cells
    # (full rows fit every member, so none is split)
    assert b.two_step_layout() == [(6, 20), (8, 21), (3, 22), (7, 23)]
    assert b.two_step_tiles() == [(80, 6, 20), (63, 8, 21), (153, 3, 22), (69, 7, 23)]
    b.step(steps)
    for k, s in enumerate(members):
        assert s.time == steps
        assert np.array_equal(s.populations().cpu().numpy(), want[k]), k
    b.set_tuning(256, 0, 16)
    with pytest.raises(vanse.VanseError) as e:
        b.two_step_layout()
    assert e.value.code == vanse.ESTATE
    b.close()
    for s in members:
        s.close()


def test_two_step_batch_single_small_member_short_segments_bitwise():
    """One 80^3 request alone (a 768-thread general tile of 7 rows: 12 tiles
    per z-segment) has 36 tiles with 32-plane segments; the batched launch
    gives it shorter ones and it still equals the solve stepped alone."""
    dtype = vanse.FP32_SHIFTED
    solo = _make_lat("D3Q19", (80, 80, 80), 0.6, 31, dtype)
    solo.step(21)
    want = solo.populations().cpu().numpy()
    solo.close()
    m = _make_lat("D3Q19", (80, 80, 80), 0.6, 31, dtype)
    b = vanse.Batch([m])
    b.set_tuning(256, vanse.TUNE_TWO_STEP, 16)
    (r, p), = b.two_step_layout()
    print("tile", r, p, flush=True)
    assert r == 7 and p in [_balanced(80, t) for t in (24, 16, 12, 8)]
    b.step(21)
    assert np.array_equal(m.populations().cpu().numpy(), want)
    b.close()
    m.close()


@pytest.mark.parametrize("dtype", [vanse.FP32_SHIFTED, vanse.FP64])
def test_uniform_batch_of_one_128_cube_takes_shorter_segments_bitwise(dtype):
    """One 128^3 solve in the batched launch takes the compile-time 128 x 4
    tile; with 64-plane segments it would have 64 tiles for 256 CUs, so its
    nz is split into 16-plane segments (256 tiles), and it still equals the
    solve stepped alone."""
    solo = _make_lat("D3Q19", (128, 128, 128), 0.6, 41, dtype)
    solo.step(13)
    want = solo.populations().cpu().numpy()
    solo.close()
    m = _make_lat("D3Q19", (128, 128, 128), 0.6, 41, dtype)
    b = vanse.Batch([m])
    b.set_tuning(256, vanse.TUNE_TWO_STEP, 16)
    assert b.two_step_layout() == [(4, 16)]
    b.step(13)
    assert np.array_equal(m.populations().cpu().numpy(), want)
    b.close()
    m.close()


# members whose full x-rows do not fit a block (FP64: 192, 257 and 360
# wide; reduced storage: 360 wide) make the batched two-step launch split
# their x-rows into segments of at most 62 columns with a halo column on each
# side (one wave per row); the other members keep full rows in the same
# launch
XT_MEMBERS = [((192, 20, 9), 0.6, 11), ((160, 13, 7), 0.8, 12), ((130, 9, 6), 0.7, 13),
              ((40, 12, 10), 0.9, 14), ((257, 5, 4), 0.66, 15), ((360, 7, 5), 0.75, 16)]


@pytest.mark.parametrize("dtype", [vanse.FP64, vanse.FP32_SHIFTED, vanse.FP16_SHIFTED,
                                   vanse.FX16_SHIFTED])
@pytest.mark.parametrize("steps,chunk", [(37, 16), (10, 0)])
def test_two_step_batch_x_split_tiles_bitwise(dtype, steps, chunk):
    print("case", dtype, steps, chunk, flush=True)
    f64 = dtype == vanse.FP64
    pre = [0, 2, 0, 4, 2, 1]
    solo = [_make(d, t, s, dtype, p) for (d, t, s), p in zip(XT_MEMBERS, pre)]
    for s in solo:
        s.step(steps)
    want = [s.populations().cpu().numpy() for s in solo]
    for s in solo:
        s.close()
    members = [_make(d, t, s, dtype, p) for (d, t, s), p in zip(XT_MEMBERS, pre)]
    b = vanse.Batch(members)
    b.set_tuning(128, vanse.TUNE_TWO_STEP, chunk)
    tiles = b.two_step_tiles()
    print("tiles", tiles, flush=True)
    want_tiles = [_xt_tile(d[0], d[1], f64) for d, _, _ in XT_MEMBERS]
    assert [(c, r) for c, r, _ in tiles] == want_tiles
    split = [c < d[0] for (c, _, _), (d, _, _) in zip(tiles, XT_MEMBERS)]
    assert split == ([True, False, False, False, True, True] if f64 else
                     [False, False, False, False, False, True])
    assert want_tiles[5] == ((60, 6) if f64 else (60, 7))
    assert [(r, p) for _, r, p in tiles] == b.two_step_layout()
    b.step(steps)
    for k, s in enumerate(members):
        assert s.time == pre[k] + steps
        assert np.array_equal(s.populations().cpu().numpy(), want[k]), k
    b.close()
    for s in members:
        s.close()
