"""Host emulation of the two-step kernel's indexing (CPU).

The two-step launch (two time levels per launch through an LDS tile that
marches in z) is only correct if every index it computes stays in bounds and
its staging buffers hold the right data when read.  This test walks every
block, loop iteration and thread of the tile scheme for many lattice shapes
and tile sizes -- general tiles (any nx, a shorter last tile in y) and the
compile-time ones -- and checks, as the kernel computes them:

* global population, phi and output addresses lie inside their arrays;
* the LDS slab: each interior cell of the tile receives each direction from
  exactly one halo cell per plane (the repeated lanes past the last halo cell
  aside), at an index inside the slab;
* the LDS phi ring of 5 planes: every read finds the plane it wants in its
  slot, written before the barrier that precedes the read;
* each destination slot of the output array is written by exactly one owning
  thread over the launch;
* the halo-wave skip (a wave collides and pushes only if its first lane is a
  real halo cell, or a compile-time constant says the whole halo slot is
  real): no real halo cell sits in a skipped wave, every slab slot is
  written by a computing wave, and a computing lane past the tile repeats a
  cell that its real lane computes in the same phase.  Nothing computed
  inside the skipped branch is carried to a later iteration (the next
  plane's loads are issued before it), so a skipped wave changes no value
  that is read.

The emulation restates the kernel's index arithmetic in numpy; it shares no
code with the HIP source.
"""
import itertools

import numpy as np
import pytest

D3Q19 = [(0,0,0),(1,0,0),(0,1,0),(0,0,1),(1,1,0),(1,-1,0),(1,0,1),(1,0,-1),(0,1,1),(0,1,-1),
         (-1,0,0),(0,-1,0),(0,0,-1),(-1,-1,0),(-1,1,0),(-1,0,-1),(-1,0,1),(0,-1,-1),(0,-1,1)]
D3Q27 = [(0,0,0)] + [c for c in itertools.product((-1,0,1), repeat=3) if c != (0,0,0) and c > (0,0,0)]
D3Q27 = D3Q27 + [tuple(-v for v in c) for c in D3Q27[1:]]


def check(nx, ny, nz, TY, SZ, lat, full=True, NT=512, TXMAX=None):
    """TXMAX: the x-split general tiles of the batched launch (tiles of
    TXMAX interior columns, a shorter last one, plus a halo column on each
    side); None or >= nx: full x-rows."""
    Q = len(lat)
    ncells = nx * ny * nz
    S = (ncells + 127) // 128 * 128
    nxy = nx * ny
    TYMAX = TY
    IPT, HPT = -(-nx * TY // NT), -(-nx * (TY + 2) // NT)
    # pert values per thread: exact for the compile-time tiles (256 x 4,
    # 256 x 2, 128 x 4 for D3Q19; 256 x 4, 256 x 2 for D3Q27), else a bound
    tiles = {(256, 4), (256, 2), (128, 4)} if Q == 19 else {(256, 4), (256, 2)}
    XT = TXMAX is not None
    xs = XT and TXMAX < nx
    compile_time = (nx, TY) in tiles and ny % TY == 0 and not XT
    NW = NT // 64
    if xs:
        # one wave per tile row of at most 64 cells: cells per thread count
        # rows per wave
        assert TXMAX + 2 <= 64
        IPT, HPT = -(-TY // NW), -(-(TY + 2) // NW)
    if compile_time:
        PPT = -(-(TY + 4) * nx // NT)
    elif XT:
        PPT = 2 * HPT
    else:
        PPT = (5 * HPT + 2) // 3
    fnxb = -(-nx // TXMAX) if xs else 1
    fnyb = -(-ny // TY) * fnxb
    nzb = -(-nz // SZ)
    tid = np.arange(NT)
    lane, wv = tid & 63, tid >> 6
    written = np.zeros((Q, ncells), np.int32)

    def wrap(v, n):
        r = np.where(v < 0, v + n, np.where(v >= n, v - n, v))
        assert np.all((r >= 0) & (r < n)), ("wrap", v, n)
        return r

    def zmod(v):
        assert np.all(np.asarray(v) >= -3 * nz)
        return (np.asarray(v) + 3 * nz) % nz

    for b in range(fnyb * nzb):
        bz = b // fnyb
        tb = b - bz * fnyb
        yb, xb = tb // fnxb, tb % fnxb
        y0 = yb * TYMAX
        x0 = xb * TXMAX if xs else 0
        TY = min(TYMAX, ny - y0)      # shorter last tile (general tiles)
        TX = min(TXMAX, nx - x0) if xs else nx
        HW, RW = (TX + 2, TX + 4) if xs else (nx, nx)
        NI, HC, PR = TX * TY, HW * (TY + 2), TY + 4
        PC = PR * RW

        def halo_x(hx):
            return wrap(x0 - 1 + hx, nx) if xs else hx

        def ring_x(c):
            return wrap(x0 - 2 + c, nx) if xs else c

        def halo_map(h):
            """(row, column, real) of each thread's halo cell in pass h."""
            if xs:
                r = wv + h * NW
                return (np.minimum(r, TY + 1), np.minimum(lane, HW - 1),
                        (lane < HW) & (r < TY + 2))
            idx = np.minimum(tid + h * NT, HC - 1)
            hr = idx // HW
            return hr, idx - hr * HW, tid + h * NT < HC

        def interior_map(k):
            """(row, column, owned) of each thread's interior cell in pass k."""
            if xs:
                rr = wv + k * NW
                return (np.minimum(rr, TY - 1), np.minimum(lane, TX - 1),
                        (lane < TX) & (rr < TY))
            cell = np.minimum(tid + k * NT, NI - 1)
            r = cell // TX
            return r, cell - r * TX, tid + k * NT < NI
        assert PC <= PPT * NT
        if xs:
            assert HW <= 64 and TY + 2 <= HPT * NW and TY <= IPT * NW
        else:
            assert NI <= IPT * NT and HC <= HPT * NT
        z0 = bz * SZ
        z1 = min(z0 + SZ, nz)
        ring = {}          # slot -> (plane, iteration written; -99 prologue)
        slot = lambda q: (q - (z0 - 2)) % 5

        def load_pert(q):
            qz = zmod(q)
            for j in range(PPT):
                idx = np.minimum(tid + j * NT, PC - 1)
                r = idx // RW
                x = ring_x(idx - r * RW)
                y = ((y0 + r - 2) % ny + ny) % ny
                a = qz * nxy + y * nx + x
                assert np.all((a >= 0) & (a < ncells)), "pert load"

        def store_pert(q, it):
            for j in range(PPT):
                idx = np.minimum(tid + j * NT, PC - 1)
                ri = slot(q) * PC + idx
                assert np.all((ri >= 0) & (ri < 5 * PC)), "ring store"
            ring[slot(q)] = (q, it)

        def ring_read(q, r, x, it, phase, want_x=None):
            """x: the ring column; want_x: the global column it must hold."""
            assert q - (z0 - 2) >= 0
            ri = (slot(q) * PR + r) * RW + x
            assert np.all((r >= 0) & (r < PR)), ("ring row", r)
            assert np.all((x >= 0) & (x < RW)), ("ring column", x)
            if want_x is not None:
                assert np.all(ring_x(x) == want_x), "ring column holds another x"
            assert np.all((ri >= 0) & (ri < 5 * PC)), "ring read"
            plane, w_it = ring[slot(q)]
            assert plane == q, ("ring holds", plane, "wanted", q)
            # halo reads need the plane written before barrier A of this
            # iteration; interior reads (after barrier B) may see this one's
            assert w_it < it or (phase == "interior" and w_it == it), (q, w_it, it, phase)

        def load_plane(p):
            pz = zmod(p)
            for h in range(HPT):
                hr, hx, _ = halo_map(h)
                x = halo_x(hx)
                y = wrap(y0 + hr - 1, ny)
                for i in range(Q):
                    a = i * S + pz * nxy + y * nx + x
                    assert np.all((a >= 0) & (a < Q * S)), "pop load"

        for q in range(z0 - 2, z0 + 1):
            load_pert(q)
            store_pert(q, -99)
        load_pert(z0 + 1)
        pending_pert = z0 + 1
        load_plane(z0 - 1)
        for p in range(z0 - 1, z1 + 1):
            pz = int(wrap(np.array(p), nz))
            slab = np.zeros((Q, NI), np.int32)
            pushed = np.zeros((Q, NI), np.int32)   # pushes by computing lanes (repeats too)
            # the last halo cell HC - 1: its halo slot and whether its wave computes
            h2_of_last = (HC - 1) // NT
            lane_last = (HC - 1) - h2_of_last * NT
            computing_last = bool((compile_time and (h2_of_last + 1) * NT <= (TYMAX + 2) * nx)
                                  or ((lane_last & ~63) + h2_of_last * NT < HC))
            store_pert(pending_pert, p)
            assert pending_pert == p + 2
            # halo phase
            for h in range(HPT):
                hr, hx, real = halo_map(h)
                x = halo_x(hx)
                c = hx + 1 if xs else x
                cm = c - 1 if xs else np.where(c == 0, nx, c) - 1
                cp = c + 1 if xs else np.where(c + 1 == nx, 0, c + 1)
                xm, xp = wrap(x - 1, nx), wrap(x + 1, nx)
                r = hr + 1
                for (qq, rr, cc, gx) in ((p, r, c, x), (p, r, cp, xp), (p, r, cm, xm),
                                         (p, r + 1, c, x), (p, r - 1, c, x), (p + 1, r, c, x),
                                         (p - 1, r, c, x)):
                    ring_read(qq, rr, cc, p, "halo", gx)
                # lanes past the last halo cell (x-split tiles: past the row
                # segment, or rows past the tile) repeat a real cell.  The
                # halo-wave skip: a wave collides and pushes only if its first
                # lane is a real halo cell (x-split tiles: its row lies in the
                # tile), or the compile-time constant FULL says every lane of
                # this halo slot is real
                FULL = compile_time and (h + 1) * NT <= (TYMAX + 2) * nx
                if xs:
                    computing = wv + h * NW < TY + 2
                else:
                    computing = FULL | ((tid & ~63) + h * NT < HC)
                if FULL:
                    assert np.all(real), "FULL with a lane past the tile"
                assert np.all(computing[real]), "a real halo cell in a skipped wave"
                # a computing lane past the tile repeats the last halo cell, which
                # its own (real) lane computes from the same inputs in this phase
                rep = computing & ~real
                if rep.any() and not XT:
                    assert computing_last, "the repeated cell is not computed"
                for i, (cx, cy, cz) in enumerate(lat):
                    rd = hr - 1 + cy
                    ok = (rd >= 0) & (rd < TY)
                    if xs:
                        xd = hx - 1 + cx           # tile column, kept inside the tile
                        ok = ok & (xd >= 0) & (xd < TX)
                        assert np.all(~ok | (x0 + xd == wrap(x + cx, nx))), "slab column"
                    else:
                        xd = wrap(x + cx, nx)
                    sidx = rd * TX + xd
                    assert np.all(~ok | ((sidx >= 0) & (sidx < NI))), "slab push"
                    np.add.at(slab[i], sidx[ok & real], 1)
                    # the x-split kernel pushes from real lanes only
                    np.add.at(pushed[i], sidx[ok & computing & (real if XT else True)], 1)
            # every interior cell receives each direction from exactly one real
            # halo cell, and every slab slot is written by a computing wave
            assert np.all(slab == 1), ("slab coverage", slab.min(), slab.max())
            assert np.all(pushed >= 1), "slab slot written by no computing wave"
            load_pert(p + 3)
            pending_pert = p + 3
            load_plane(p + 1)
            z = max(p - 1, z0)
            assert 0 <= z < nz
            for k in range(IPT):
                r, cx_, owned = interior_map(k)
                own = owned & (p > z0)
                cell = r * TX + cx_
                assert np.all((cell >= 0) & (cell < NI)), "slab read"
                x = x0 + cx_
                y = y0 + r
                assert np.all((y < ny) & (x < nx))
                c = cx_ + 2 if xs else x
                cm = c - 1 if xs else np.where(c == 0, nx, c) - 1
                cp = c + 1 if xs else np.where(c + 1 == nx, 0, c + 1)
                xm, xp = wrap(x - 1, nx), wrap(x + 1, nx)
                rr = r + 2
                for (qq, r2, cc, gx) in ((z, rr, c, x), (z, rr, cp, xp), (z, rr, cm, xm),
                                         (z, rr + 1, c, x), (z, rr - 1, c, x), (z + 1, rr, c, x),
                                         (z - 1, rr, c, x)):
                    ring_read(qq, r2, cc, p, "interior", gx)
                for i, (cx, cy, cz) in enumerate(lat):
                    yd, zd, xd = wrap(y + cy, ny), int(wrap(np.array(z + cz), nz)), wrap(x + cx, nx)
                    a = zd * nxy + yd * nx + xd
                    assert np.all((a >= 0) & (a < ncells))
                    np.add.at(written[i], a[own], 1)
        if not full and b > 3:
            break
    if full:
        assert np.all(written == 1), ("coverage", written.min(), written.max())
    return True



# (nx, ny, nz, rows per tile, planes per segment)
CASES = [(64, 8, 6, 1, 4), (64, 8, 6, 2, 32), (64, 8, 6, 4, 1), (64, 8, 6, 8, 3), (128, 4, 5, 2, 2),
         (64, 2, 1, 2, 8), (64, 1, 2, 1, 1), (192, 6, 7, 3, 5), (256, 4, 9, 4, 4), (128, 12, 3, 6, 2),
         (64, 3, 2, 3, 1), (64, 1, 1, 1, 1), (128, 2, 3, 1, 7), (256, 8, 3, 2, 64), (256, 8, 5, 4, 64),
         # general tiles
         (48, 10, 7, 4, 3), (33, 17, 5, 5, 2), (96, 7, 6, 3, 4), (7, 5, 3, 2, 1), (1, 1, 1, 1, 1),
         (64, 9, 4, 4, 8), (130, 3, 2, 2, 2), (40, 6, 5, 4, 3), (17, 3, 2, 2, 1), (17, 13, 11, 13, 11),
         (5, 64, 7, 64, 7), (191, 9, 5, 2, 32), (33, 40, 6, 15, 32)]


@pytest.mark.parametrize("lat", ["D3Q19", "D3Q27"])
@pytest.mark.parametrize("case", CASES)
def test_two_step_tile_indexing(case, lat):
    assert check(*case, D3Q19 if lat == "D3Q19" else D3Q27)


@pytest.mark.parametrize("case", [(256, 256, 256, 4, 64), (256, 256, 256, 2, 64),
                                  (128, 128, 128, 4, 8), (512, 64, 16, 2, 8)])
def test_two_step_tile_indexing_full_size_first_blocks(case):
    """The first blocks of full-size launches (the 256^3 benchmark shapes)."""
    assert check(*case, D3Q19, full=False)


@pytest.mark.parametrize("case", [(128, 8, 20, 4, 16), (256, 4, 130, 2, 128),
                                  (128, 128, 128, 4, 16)])
def test_two_step_benchmarked_512_thread_tiles(case):
    """The compile-time 128 x 4 and 256 x 2 tiles of the benchmarked launches
    (128^3 FP64 with 16-plane segments; 256^3 FP64 with 128-plane segments),
    with the halo-wave skip."""
    assert check(*case, D3Q19, full=case[0] * case[1] * case[2] < 2_000_000)


@pytest.mark.parametrize("case", [(256, 8, 5, 4, 64), (256, 4, 9, 4, 4), (256, 12, 3, 4, 2)])
def test_two_step_tile_indexing_1024_threads(case):
    """The 256 x 4 tile in 1024-thread blocks (one interior, two halo cells
    per thread, the second halo cell of half the threads past the tile)."""
    assert check(*case, D3Q19, NT=1024)
    assert check(256, 256, 256, 4, 64, D3Q19, full=False, NT=1024)


# x-split general tiles of the batched launch: (nx, ny, nz, rows, planes, cols)
XT_CASES = [(130, 9, 6, 6, 5, 44), (129, 7, 5, 10, 2, 43), (100, 12, 3, 13, 2, 34),
            (8, 5, 3, 2, 2, 3), (61, 17, 4, 14, 3, 31), (70, 3, 2, 3, 2, 62),
            # members that keep full rows in a launch with x-split members
            (64, 8, 4, 8, 4, 64), (33, 5, 4, 5, 2, 33), (40, 12, 10, 12, 5, 40),
            (96, 9, 3, 8, 3, 96),
            # the tiles the batched launch picks: FP64 192, 257 wide (6 rows);
            # reduced storage 360 wide (14 rows), and 192 wide
            (192, 20, 9, 6, 4, 48), (257, 5, 4, 5, 4, 52), (360, 7, 5, 7, 2, 60),
            (360, 30, 3, 14, 3, 60), (192, 20, 9, 14, 4, 48)]


# general tiles of batches of narrow members: 768-thread blocks, one
# interior and one halo cell per thread, rows = 768 / nx - 2 (at most ny):
# (nx, ny, nz, rows, planes)
GEN768_CASES = [(32, 32, 5, 22, 2), (48, 48, 4, 14, 3), (64, 64, 3, 10, 3), (96, 96, 3, 6, 2),
                (17, 13, 11, 13, 6), (80, 80, 3, 7, 2), (67, 13, 4, 9, 4), (5, 64, 7, 64, 3),
                (33, 40, 3, 21, 2)]


@pytest.mark.parametrize("case", GEN768_CASES)
def test_two_step_general_tile_indexing_768_threads(case):
    nx, ny, nz, rows, planes = case
    assert rows == min(768 // nx - 2, ny)
    assert check(nx, ny, nz, rows, planes, D3Q19, full=True, NT=768)


@pytest.mark.parametrize("lat", ["D3Q19"])
@pytest.mark.parametrize("case", XT_CASES)
def test_two_step_x_split_tile_indexing(case, lat):
    """Tiles of `cols` interior columns with a halo column on each side (the
    last tile of a row shorter), and members of an x-split batch that keep
    full rows (cols >= nx)."""
    nx, ny, nz, rows, planes, cols = case
    assert check(nx, ny, nz, rows, planes, D3Q19, TXMAX=cols)


def _chosen_tiles(nx, ny, f64):
    """The batched launch's tile for a member of width nx: (threads, rows,
    columns) of the 512-thread general tile, the 768-thread one (reduced
    storage, nx <= 96) and the x-split launch's tile, as the host chooses
    them (batch_fused_rows, batch_xt_tile)."""
    out = []
    r512 = min(512 // nx - 2 if f64 else min(512 // nx, 1024 // nx - 2), ny)
    if r512 >= 1:
        out.append((512, r512, nx))
    if not f64 and nx <= 96:
        r768 = min(768 // nx - 2, ny)
        if r768 >= 1:
            out.append((768, r768, nx))
    per = 1 if f64 else 2
    if nx > (170 if f64 else 341) and nx > 62:
        k = -(-nx // 62)
        out.append((512, min(per * 8 - 2, ny), -(-nx // k)))
    else:
        rf = min(per * 512 // nx - 2, ny)
        if rf >= 1:
            out.append((512, rf, -1))   # full rows inside an x-split launch
    return out


def test_random_sizes_tile_indexing():
    """Every tile the batched launch can choose, for seeded random member
    sizes, keeps every access in bounds and covers every output once."""
    rng = np.random.default_rng(2208)
    for _ in range(40):
        f64 = bool(rng.integers(0, 2))
        nx = int(rng.integers(3, 420))
        ny = int(rng.integers(1, 24))
        nz = int(rng.integers(1, 6))
        for nt, rows, cols in _chosen_tiles(nx, ny, f64):
            planes = int(rng.integers(1, nz + 1))
            txmax = None if cols == nx else (nx if cols < 0 else cols)
            assert check(nx, ny, nz, rows, planes, D3Q19, full=True, NT=nt, TXMAX=txmax), \
                (nx, ny, nz, rows, planes, nt, cols)

