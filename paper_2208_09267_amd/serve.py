"""Continuous-batching request loop for VANSE lattice Boltzmann solves on one
GPU.

Requests (a workload: size, tau, phi, steps) arrive over time.  The loop
admits them first-come-first-served as device memory (an HBM budget) and a
cap on the cells in flight allow, keeps every admitted solve's populations
resident on the device, and advances ALL admitted solves together with the
batched launch (one kernel per time step covering every solve; chunks of
steps replay a captured graph).  A solve that reaches its step count is
retired at the next chunk boundary: its moments are copied to the host and
its memory is freed, which lets queued requests in.  While the head of the
queue does not fit (or no request is left to arrive), nothing can join
before the next retirement, so the batch runs straight to it without
returning to the host between chunks.  Requests that arrive
while others are on the GPU therefore overlap with them on the device.
Because the per-cell arithmetic of the batched launch does not depend on
the other members, every result is bitwise identical alone and in the mix.

Latency = arrival time -> the time the solve's moments (rho, p, u in FP64)
have been copied into host memory.  The copy goes to a pinned staging buffer
that the loop reuses; keep_fields=True also hands each result its own numpy
arrays.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import vanse
from . import workloads as W

_Q = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}
_ELEM = {vanse.FP64: 8, vanse.FP32_SHIFTED: 4, vanse.FP16_SHIFTED: 2, vanse.FX16_SHIFTED: 2}
_PERT = {vanse.FP64: 8, vanse.FP32_SHIFTED: 4, vanse.FP16_SHIFTED: 4, vanse.FX16_SHIFTED: 4}


def state_bytes(lattice: str, dims, dtype: int, two_step: bool = False) -> int:
    """Device bytes one solve holds (the layout vanse_create allocates:
    Q population planes and one phi plane of stride round_up(ncells, 128),
    plus the reduction scratch; with two_step, on a 3-D lattice, the second
    population array of the two-step launch)."""
    n = int(np.prod(dims))
    stride = (n + 127) // 128 * 128
    pop = _Q[lattice] * stride * _ELEM[dtype]
    if two_step and lattice != "D2Q9":
        pop *= 2
    return pop + stride * _PERT[dtype] + 8 * (7 * 1024 + 64)


def admit_count(queue_bytes: Sequence[int], queue_cells: Sequence[int], used_bytes: int,
                active_cells: int, n_active: int, budget_bytes: int, cell_cap: int,
                max_active: int) -> int:
    """How many requests at the head of the FCFS queue to admit now.

    A request is admitted while its state fits in the remaining HBM budget,
    the cells in flight stay within cell_cap (enough cells to saturate the
    GPU; more only stretches every solve) and the member count stays within
    max_active.  The head always goes first: no request overtakes another.
    When nothing is active, the head is admitted even above cell_cap (but
    never above the budget), so one large request cannot starve."""
    k = 0
    for b, c in zip(queue_bytes, queue_cells):
        if used_bytes + b > budget_bytes or n_active + 1 > max_active:
            break
        if n_active > 0 and active_cells + c > cell_cap:
            break
        used_bytes += b
        active_cells += c
        n_active += 1
        k += 1
    return k


def steps_until_host(min_remaining: int, chunk: int, queue_waiting: bool,
                     arrivals_left: bool) -> int:
    """Steps the batch advances before the loop looks at the host again.

    The first retirement comes after min_remaining steps.  While requests may
    still arrive and nothing is queued, the loop stops at the next chunk
    boundary so that a new arrival joins promptly.  Otherwise nothing can join
    before that retirement (the queue head does not fit, or no request is left
    to arrive), so the batch runs straight to it."""
    if not queue_waiting and arrivals_left:
        return min(min_remaining, chunk)
    return min_remaining


def tune_trial_steps(min_remaining: int, longest: int = 16) -> int:
    """Steps per autotuner trial that keep all of its real steps (at most
    10 t + 9 for t steps per trial) within the fewest steps any member has
    left; 0 when not even a one-step trial fits."""
    return max(0, min(longest, (min_remaining - 9) // 10))


def retune(prev_trial: int, trial: int, longest: int = 16) -> bool:
    """Whether to autotune a size class now: it has no choice yet
    (prev_trial 0) and a trial fits, or its choice came from trials shorter
    than the longest and a longest trial fits now (short trials do not
    resolve launches a few percent apart)."""
    if trial < 1:
        return False
    return prev_trial == 0 or (prev_trial < longest and trial >= longest)


@dataclasses.dataclass
class Result:
    rid: int
    name: str
    arrival: float
    admit: float = float("nan")
    finish: float = float("nan")
    steps: int = 0
    cells: int = 0
    error: Optional[str] = None
    rho: Optional[np.ndarray] = None
    p: Optional[np.ndarray] = None
    u: Optional[np.ndarray] = None

    @property
    def latency(self):
        return self.finish - self.arrival


@dataclasses.dataclass
class _Active:
    rid: int
    work: W.Workload
    solver: vanse.Solver
    remaining: int
    result: Result


class Server:
    """Continuous-batching loop.  budget_bytes: HBM the resident states may
    use; cell_cap: cells in flight; chunk: steps between admissions (and per
    captured graph); two_step: let the batch use the two-step launch (its
    second population arrays are counted in the budget; a request admitted
    while the batch sits at an odd level takes one step alone first, so all
    members share the parity the two-step launch needs)."""

    def __init__(self, budget_bytes=200e9, cell_cap=40_000_000, max_active=4096, chunk=16,
                 dtype=vanse.FP32_SHIFTED, keep_fields=False, autotune=True, log=None,
                 two_step=True):
        self.budget = int(budget_bytes)
        self.cell_cap = int(cell_cap)
        self.max_active = int(max_active)
        self.chunk = int(chunk)
        self.dtype = dtype
        self.keep_fields = keep_fields
        self.autotune = autotune
        self.two_step = two_step
        self.log = log
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stats = collections.Counter()
        self.time = collections.Counter()  # host seconds per loop phase
        # default batched launch, and the autotuned one per size class
        self.tuning = (256, vanse.TUNE_TWO_STEP if two_step else 0)
        self._tuned = {}
        self._host = torch.empty(0, dtype=torch.float64)  # pinned staging of the moments

    def _to_host(self, solver) -> Tuple[np.ndarray, ...]:
        """Copy the solve's moments into the pinned staging buffer (grown
        when needed, then reused) and wait for the copy.  Returns (rho, p, u)
        views into that buffer, valid until the next call."""
        fields = solver.moments()
        total = sum(t.numel() for t in fields)
        if self._host.numel() < total:
            self._host = torch.empty(max(total, self._host.numel() * 3 // 2),
                                     dtype=torch.float64, pin_memory=True)
        views, off = [], 0
        for t in fields:
            dst = self._host[off:off + t.numel()].view(t.shape)
            dst.copy_(t, non_blocking=True)
            views.append(dst)
            off += t.numel()
        torch.cuda.current_stream().synchronize()
        return tuple(v.numpy() for v in views)

    def _bytes(self, work: W.Workload) -> int:
        return state_bytes(work.lattice, work.dims, self.dtype, self.two_step)

    def _start(self, rid, work: W.Workload, now) -> Tuple[Optional[_Active], Result]:
        res = Result(rid, work.name, arrival=now, steps=work.steps, cells=work.ncells)
        try:
            s = vanse.Solver(work.lattice, work.dims, work.tau, self.dtype)
            try:
                s.set_porosity(work.eps_mean, W.fourier_eps_device(work.dims, work.seed, self.device),
                               work.period, work.quad_axes)
                s.set_force(work.force)
                d = 2 if work.lattice == "D2Q9" else 3
                s.init(None, W.taylor_green_device(work.dims, work.tgv_amp, self.device, d))
            except Exception:
                s.close()
                raise
        except (vanse.VanseError, ValueError) as e:
            res.error = str(e)
            return None, res
        return _Active(rid, work, s, work.steps, res), res

    def run(self, arrivals: Sequence[Tuple[float, W.Workload]], realtime=True) -> List[Result]:
        """Serve `arrivals` (time in seconds from start, workload), in
        arrival order.  realtime=False admits every request at time 0 (an
        offline batch).  Returns one Result per request, in arrival order."""
        arrivals = sorted(enumerate(arrivals), key=lambda r: r[1][0])
        clock = time.perf_counter
        t0 = clock()
        queue = collections.deque()  # (rid, arrival, workload)
        queued_bytes = collections.deque()  # state bytes and cells of the queued requests
        queued_cells = collections.deque()
        active: List[_Active] = []
        results = {}
        batch = None
        dirty = False
        block, flags = self.tuning  # the batched launch in effect
        i = 0
        used = 0
        while i < len(arrivals) or queue or active:
            now = clock() - t0
            tadm = clock()
            while i < len(arrivals) and (not realtime or arrivals[i][1][0] <= now):
                rid, (ta, work) = arrivals[i]
                queue.append((rid, ta if realtime else 0.0, work))
                queued_bytes.append(self._bytes(work))
                queued_cells.append(work.ncells)
                i += 1
            k = admit_count(queued_bytes, queued_cells, used, sum(a.work.ncells for a in active),
                            len(active), self.budget, self.cell_cap, self.max_active)
            if k == 0 and not active and queue:
                # the head can never fit: fail it rather than wait forever
                rid, ta, work = queue.popleft()
                queued_bytes.popleft()
                queued_cells.popleft()
                res = Result(rid, work.name, ta, steps=work.steps, cells=work.ncells,
                             error="request needs %d bytes, over the HBM budget"
                                   % self._bytes(work))
                res.finish = clock() - t0
                results[rid] = res
                continue
            for _ in range(k):
                rid, ta, work = queue.popleft()
                queued_bytes.popleft()
                queued_cells.popleft()
                act, res = self._start(rid, work, ta)
                res.admit = clock() - t0
                if act is None:
                    res.finish = res.admit
                    results[rid] = res
                    self.stats["failed"] += 1
                    continue
                if active and active[0].solver.time % 2 and act.remaining > 0:
                    act.solver.step(1)  # join at the batch's parity
                    act.remaining -= 1
                active.append(act)
                used += self._bytes(work)
                dirty = True
            self.time["admit"] += clock() - tadm
            if not active:
                if i < len(arrivals) and realtime:
                    time.sleep(max(0.0, arrivals[i][1][0] - (clock() - t0)))
                continue
            if dirty:
                tr = clock()
                if batch is None:
                    batch = vanse.Batch([a.solver for a in active])
                else:
                    batch.update([a.solver for a in active])
                block, flags = self.tuning
                if self.autotune:
                    # the library caches its choice per size class (log2 of the
                    # cells); a class without a choice yet is tuned when the
                    # trials fit, otherwise it takes the default launch
                    cls = sum(a.work.ncells for a in active).bit_length() - 1
                    prev = self._tuned.get(cls)
                    block, flags = prev[:2] if prev else self.tuning
                    # trial steps are real steps: keep them within every member's count
                    # (6 single-step trials of t, one aligning step, then twice a
                    # two-step trial of t rounded up to a multiple of 4 and a
                    # single-step one of t rounded up to even: at most 10 t + 9
                    # steps).  Longer trials resolve launches that differ by a few
                    # percent on small batches, where a trial of a few steps lasts
                    # well under a millisecond.
                    trial = tune_trial_steps(min(a.remaining for a in active))
                    if retune(prev[2] if prev else 0, trial):
                        block, flags, ran = batch.autotune(trial)
                        self._tuned[cls] = (block, flags, trial)
                        for a in active:
                            a.remaining -= ran
                if not self.two_step:
                    flags &= ~vanse.TUNE_TWO_STEP
                batch.set_tuning(block, flags, self.chunk)
                dirty = False
                self.stats["rebuilds"] += 1
                self.time["rebuild"] += clock() - tr
            ts = clock()
            step = steps_until_host(min(a.remaining for a in active), self.chunk, bool(queue),
                                    i < len(arrivals))
            if step > 0:
                batch.step(step)
                for a in active:
                    a.remaining -= step
                self.stats["chunks"] += 1
                # batch steps and lattice updates taken under a two-step or a
                # single-step tuning
                kind = "two_step" if self.two_step and flags & vanse.TUNE_TWO_STEP else "single_step"
                self.stats["steps_" + kind + "_tuning"] += step
                self.stats["lups_" + kind + "_tuning"] += step * sum(a.work.ncells for a in active)
            torch.cuda.current_stream().synchronize()
            self.time["step"] += clock() - ts
            done = [a for a in active if a.remaining <= 0]
            if done:
                tr = clock()
                # the batch keeps the retired members' pointers until the next
                # update, but it is not stepped before that
                dirty = True
                for a in done:
                    rho, p, u = self._to_host(a.solver)
                    a.result.finish = clock() - t0   # its moments are in host memory
                    if self.keep_fields:
                        a.result.rho, a.result.p, a.result.u = rho.copy(), p.copy(), u.copy()
                    results[a.rid] = a.result
                    used -= self._bytes(a.work)
                    a.solver.close()
                    if self.log:
                        self.log(a.result)
                active = [a for a in active if a.remaining > 0]
                self.time["retire"] += clock() - tr
        if batch is not None:
            batch.close()
        return [results[r] for r in sorted(results)]


def summarize(results: Sequence[Result], wall: float):
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.array([float("nan")])
    lups = sum(r.cells * r.steps for r in ok)
    return {"requests": len(results), "completed": len(ok), "failed": len(results) - len(ok),
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_max_s": float(lat.max()), "makespan_s": wall,
            "aggregate_mlups": lups / wall / 1e6 if wall > 0 else float("nan")}
