#!/usr/bin/env python3
"""Throughput of the fused VANSE lattice Boltzmann step on one MI355X.

Workload (the headline configuration): D3Q19, 256^3 periodic, tau = 0.55,
phi(x, t_n) = 0.75 + cos(2 pi n / 1000) * dphi(x) with dphi the seeded sum of
8 Fourier modes (seed 1), Taylor-Green initial velocity of amplitude 0.02,
rho = 1.  Storage variants: FP32 shifted populations (headline), FP64, FP16
shifted and FX16 shifted (16-bit fixed point).  One "step" is one full time step of the whole lattice; the
state is resident in HBM before timing starts.

Prints ONE JSON line (rank 0).  `value` is the headline variant's MLUPS;
`roofline` describes the kernel that runs the steps (the single-step kernel,
or the two-step kernel when the autotuner picks it) against the 8 TB/s HBM
peak using its algorithmic bytes per launch: every population loaded once and
stored once plus one phi value per cell (a two-step launch does two lattice
updates per cell for those bytes); `cpu_baseline` times the FP64 CPU oracle
on a bounded number of steps of the same workload on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline, D3Q19 256³ FP64 vs FP32-shifted; p50/p99 solve latency"
PEAK_HBM_GBS = 8000.0
# algorithmic bytes per cell and launch: Q loads + Q stores + one phi value
# (one lattice update per cell for the single-step kernel, two for the
# two-step kernel)
BYTES_PER_PASS = {"fp64": 19 * 8 * 2 + 8, "fp32_shifted": 19 * 4 * 2 + 4,
                  "fp16_shifted": 19 * 2 * 2 + 4, "fx16_shifted": 19 * 2 * 2 + 4}
DTYPE_NAME = {"fp64": "f64", "fp32_shifted": "f32", "fp16_shifted": "f32", "fx16_shifted": "f32"}
MODE_NAME = {"fp64": "FP64", "fp32_shifted": "FP32_SHIFTED", "fp16_shifted": "FP16_SHIFTED",
             "fx16_shifted": "FX16_SHIFTED"}


def kernel_name(variant, rows, lattice="D3Q19"):
    """Label of the kernel a launch shape runs (two-step rows 0: single step);
    the same labels key the committed counter record."""
    from paper_2208_09267_amd.rocprof_summary import kernel_label
    mode = {"fp64": 0, "fp32_shifted": 1, "fp16_shifted": 2, "fx16_shifted": 3}[variant]
    return kernel_label("fused2_kernel" if rows else "step_kernel", lattice, mode, rows or None)


def kernel_source_hash():
    from paper_2208_09267_amd.rocprof_summary import kernel_source_hash as h
    return h()


def measured_traffic(variant, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_d3q19_256.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else round(k["bytes_per_launch"])


# launch shapes the autotuner picks for this workload on MI355X (used with
# --fixed-launch, e.g. under a counter profiler that perturbs timing)
# (tile_x, tile_y, flat, two-step rows, two-step planes)
FIXED_LAUNCH = {"fp32_shifted": (1024, 1, True, 4, 64), "fp64": (512, 1, True, 2, 128),
                "fp16_shifted": (256, 4, False, 4, 64), "fx16_shifted": (256, 4, False, 4, 64)}
SINGLE_LAUNCH = {"fp32_shifted": (1024, 1, True, 0, 0), "fp64": (512, 1, True, 0, 0),
                 "fp16_shifted": (256, 4, False, 0, 0), "fx16_shifted": (256, 4, False, 0, 0)}


def gpu_variant(variant, w, pert_t, u0_t, steps, warmup, fixed_launch=False):
    """Time `steps` steps of one storage variant.  fixed_launch: False =
    autotuned shape; True = the recorded shape of FIXED_LAUNCH; a tuple =
    that shape (tile_x, tile_y, flat, two-step rows, two-step planes)."""
    import torch

    from paper_2208_09267_amd import vanse

    s = vanse.Solver(w.lattice, w.dims, w.tau, vanse.DTYPES[variant])
    s.set_porosity(w.eps_mean, pert_t, w.period, w.quad_axes)
    s.set_force(w.force)
    s.init(None, u0_t)
    if fixed_launch:
        shape = FIXED_LAUNCH[variant] if fixed_launch is True else fixed_launch
        tile_x, tile_y, flat, rows, planes = shape
        flags = 4 if flat else 0
        s.set_tuning(tile_x, flags)
        s.set_tile(tile_x, tile_y)
        s.set_fused(rows, planes)
        fused = (rows, planes)
        ran = 0
    else:
        # warm-up: the autotuner's trial steps are real (untimed) steps
        L = s.autotune(8)  # real steps: they count as warm-up
        tile_x, tile_y, flags, ran = L.tile_x, L.tile_y, L.flags, L.steps_run
        fused = (L.fused_rows, L.fused_planes)
    two_step = fused[0] > 0
    extra = max(0, warmup - ran)
    if two_step and (s.time + extra) % 2:
        extra += 1  # start the timed region at an even level: two-step launches only
    s.step(extra)
    if two_step and steps % 2:
        steps += 1
    torch.cuda.synchronize()
    # the events are recorded on torch's current stream, which the solver launches on
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    s.step(steps)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    mass = s.diagnostics()[0]
    s.close()
    ms_step = ms / steps
    per_launch = 2 if two_step else 1
    launch_ms = ms_step * per_launch
    mlups = w.ncells * steps / (ms / 1e3) / 1e6
    bytes_launch = BYTES_PER_PASS[variant] * w.ncells
    gbs = bytes_launch / (launch_ms / 1e3) / 1e9
    eff = BYTES_PER_PASS[variant] * mlups * 1e6 / 1e9
    launch = {"tile_x": tile_x, "tile_y": tile_y, "flat": bool(flags & 4),
              "two_step_rows": fused[0], "two_step_planes": fused[1]}
    return {"mlups": mlups, "ms_per_step": ms_step, "ms_per_launch": launch_ms,
            "steps_per_launch": per_launch, "wall_s": wall, "gb_s": gbs,
            "frac_hbm": gbs / PEAK_HBM_GBS, "bytes_per_launch": bytes_launch,
            "bytes_per_lup": BYTES_PER_PASS[variant] / per_launch,
            "effective_gb_s": eff, "effective_frac": eff / PEAK_HBM_GBS,
            "kernel": kernel_name(variant, fused[0]), "mass": mass, "launch": launch,
            "steps": steps}


Q_OF = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}
ELEM = {"fp64": (8, 8), "fp32_shifted": (4, 4), "fp16_shifted": (2, 4), "fx16_shifted": (2, 4)}


def solo_run(w, variant, steps, warmup=30):
    """One solve of workload w in storage `variant`, in the launch the
    autotuner picks (its trial steps are real steps and count as warm-up):
    MLUPS and the roofline of the launched kernel."""
    import numpy as np
    import torch

    from paper_2208_09267_amd import vanse

    dev = torch.device("cuda", 0)
    q = Q_OF[w.lattice]
    e, pe = ELEM[variant]
    bpl = q * e * 2 + pe
    s = vanse.Solver(w.lattice, w.dims, w.tau, vanse.DTYPES[variant])
    s.set_porosity(w.eps_mean, torch.from_numpy(w.eps_pert()).to(dev), w.period, w.quad_axes)
    s.set_force(w.force)
    s.init(None, torch.from_numpy(np.ascontiguousarray(w.u0())).to(dev))
    L = s.autotune(4)
    extra = max(0, warmup - L.steps_run)
    if L.fused_rows and (s.time + extra) % 2:
        extra += 1
    s.step(extra)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    s.close()
    per_launch = 2 if L.fused_rows else 1
    gbs = bpl * w.ncells / (ms * per_launch / 1e3) / 1e9
    return {"mlups": round(w.ncells / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms, 5),
            "kernel": kernel_name(variant, L.fused_rows, w.lattice),
            "bytes_per_lup": bpl / per_launch, "gb_s": round(gbs, 1),
            "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
            "effective_frac_single_step_bytes":
                round(bpl * w.ncells / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
            "launch": {"tile_x": L.tile_x, "tile_y": L.tile_y, "flat": bool(L.flags & 4),
                       "two_step_rows": L.fused_rows, "two_step_planes": L.fused_planes}}


def d3q27_run(steps=200, warmup=30):
    """The paper's own 3-D lattice (D3Q27, Table 2) on the same 256^3
    workload: FP64 and FP32 shifted."""
    import dataclasses

    from paper_2208_09267_amd import workloads as W

    w = dataclasses.replace(W.d3q19_256(), lattice="D3Q27")
    return {v: solo_run(w, v, steps, warmup) for v in ("fp64", "fp32_shifted")}


def small_configs_run():
    """The two smaller single-solve workloads, FP64: D2Q9 64^2 (1000 steps;
    4096 cells, so launch-bound: context only) and D3Q19 128^3 (1000 steps;
    its 319 MB state partly stays in the 256 MB last-level cache)."""
    from paper_2208_09267_amd import workloads as W

    return {"d2q9_64": dict(solo_run(W.d2q9_64(), "fp64", 1000), workload="D2Q9 64^2 tau 0.8"),
            "d3q19_128": dict(solo_run(W.d3q19_128(), "fp64", 1000),
                              workload="D3Q19 128^3 tau 0.6")}


def batched_run(ws=None, steps=500, trial=5, workload=None):
    """Independent D3Q19 solves, FP32 shifted, advanced together by the
    batched launch (default: the 64 solves with edges 32/48/64/96, tau in
    [0.55, 1], own seeded phi each); the launch shape comes from the
    autotuner, whose trial steps are real steps and are included in the run.
    Returns aggregate throughput of the steps after tuning."""
    import numpy as np
    import torch

    from paper_2208_09267_amd import vanse
    from paper_2208_09267_amd import workloads as W

    if ws is None:
        ws = W.batched_64()
        workload = ("64 D3Q19 solves, edges uniform in {32,48,64,96}, tau U[0.55,1.0], "
                    "seeded phi per solve, FP32 shifted, %d steps each" % steps)
    dev = torch.device("cuda", 0)
    solvers = []
    for w in ws:
        s = vanse.Solver(w.lattice, w.dims, w.tau, vanse.FP32_SHIFTED)
        s.set_porosity(w.eps_mean, torch.from_numpy(w.eps_pert()).to(dev), w.period)
        s.init(None, torch.from_numpy(np.ascontiguousarray(w.u0())).to(dev))
        solvers.append(s)
    b = vanse.Batch(solvers)
    block, flags, run = b.autotune(trial)
    timed = steps - run
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(timed)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cells = sum(w.ncells for w in ws)
    assert all(s.time == steps for s in solvers)
    b.close()
    for s in solvers:
        s.close()
    gbs = BYTES_PER_PASS["fp32_shifted"] * cells * timed / (ms / 1e3) / 1e9
    return {"workload": workload,
            "total_cells": cells, "steps_timed": timed, "autotune_steps": run,
            "launch": {"block": block, "nontemporal": bool(flags & 1),
                       "two_step": bool(flags & vanse.TUNE_TWO_STEP), "graph_chunk": 16},
            "mlups": round(cells * timed / (ms / 1e3) / 1e6, 1),
            "ms_per_step": round(ms / timed, 5),
            # bytes a one-step-per-pass kernel would move for the same throughput
            "effective_gb_s_single_step_bytes": round(gbs, 1),
            "effective_frac_single_step_bytes": round(gbs / PEAK_HBM_GBS, 4)}


def batched_256_run(count=4, steps=200):
    """The batched launch at the headline size: `count` D3Q19 256^3 solves
    (own tau and seeded phi each), FP32 shifted."""
    from paper_2208_09267_amd import workloads as W
    return batched_run(W.batched_256(count=count), steps=steps, trial=5,
                       workload="%d D3Q19 256^3 solves, tau U[0.55,1.0], seeded phi per solve, "
                                "FP32 shifted, %d steps each" % (count, steps))


def _solve_fields(w, dtype, progress=None):
    """Run workload w for w.steps steps in the given storage mode and return
    (rho, p, u) as FP64 CUDA tensors."""
    import numpy as np
    import torch

    from paper_2208_09267_amd import vanse

    dev = torch.device("cuda", 0)
    s = vanse.Solver(w.lattice, w.dims, w.tau, dtype)
    s.set_porosity(w.eps_mean, torch.from_numpy(w.eps_pert()).to(dev), w.period)
    s.init(None, torch.from_numpy(np.ascontiguousarray(w.u0())).to(dev))
    done = 0
    while done < w.steps:
        k = min(1000, w.steps - done)
        s.step(k)
        done += k
        if progress:
            torch.cuda.synchronize()
            print("# %s: %d/%d steps" % (progress, done, w.steps), file=sys.stderr, flush=True)
    rho, p, u = s.moments()
    torch.cuda.synchronize()
    s.close()
    return rho, p, u


def precision_study():
    """Error of the FP32-, FP16- and FX16-shifted storage modes against the FP64
    path (which matches the CPU oracle to <= 1e-11) on the D3Q19 256^3
    workload after 2000 steps, next to the FP64 discretisation error at the
    same resolution, estimated against a 512^3 FP64 run of the same physical
    problem under diffusive scaling (tau fixed, dt ~ dx^2: 8000 steps, phi
    period 4000 steps, Taylor-Green amplitude 0.01; u compared as u_256 vs
    2 u_512, rho and p deviations from their means as q_256 vs 4 q_512, at
    the coincident nodes)."""
    import dataclasses

    import torch

    from paper_2208_09267_amd import vanse
    from paper_2208_09267_amd import workloads as W

    w = W.d3q19_256()
    n = w.dims[0]
    ref = {}
    for name, dt in (("fp64", vanse.FP64), ("fp32_shifted", vanse.FP32_SHIFTED),
                     ("fp16_shifted", vanse.FP16_SHIFTED), ("fx16_shifted", vanse.FX16_SHIFTED)):
        ref[name] = _solve_fields(w, dt, progress=name)
    w2 = dataclasses.replace(w, name="D3Q19 512^3 reference", dims=(2 * n,) * 3,
                             steps=4 * w.steps, period=4 * w.period, tgv_amp=w.tgv_amp / 2)
    r2, p2, u2 = _solve_fields(w2, vanse.FP64, progress="fp64 512^3")

    def inject(a, comps=None):
        g = a.view(-1, 2 * n, 2 * n, 2 * n) if comps else a.view(2 * n, 2 * n, 2 * n)
        g = g[..., ::2, ::2, ::2]
        return g.reshape(comps, -1) if comps else g.reshape(-1)

    r64, p64, u64 = ref["fp64"]
    disc = {"rho": (r64 - r64.mean()) - 4.0 * (inject(r2) - r2.mean()),
            "p": (p64 - p64.mean()) - 4.0 * (inject(p2) - p2.mean()),
            "u": (u64 - 2.0 * inject(u2, 3)).norm(dim=0)}
    del r2, p2, u2

    def norms(d):
        return {"L2": float(d.pow(2).mean().sqrt()), "Linf": float(d.abs().max())}

    out = {"workload": w.name, "steps": w.steps,
           "reference": "GPU FP64 (matches the CPU oracle to <= 1e-11 relative Linf)",
           "discretisation": {k: norms(v) for k, v in disc.items()}, "modes": {}}
    gold = os.path.join(ROOT, "tests", "golden", "d3q19_256.npz")
    if os.path.exists(gold):
        import numpy as np

        g = np.load(gold)
        cells = torch.from_numpy(g["cells"]).cuda()
        vs = {}
        for name, (r, p, u) in ref.items():
            vs[name] = {"rho": float((r[cells].cpu().numpy() - g["rho"]).__abs__().max()),
                        "p": float((p[cells].cpu().numpy() - g["p"]).__abs__().max()),
                        "u": float((u[:, cells].cpu().numpy() - g["u"]).__abs__().max())}
        out["vs_cpu_oracle_samples_linf"] = {
            "cells": int(len(g["cells"])), "oracle_field_linf": {"rho": float(g["norms"][0]),
                                                                 "p": float(g["norms"][1]),
                                                                 "u": float(g["norms"][2])},
            "abs_error": vs}
    for name in ("fp32_shifted", "fp16_shifted", "fx16_shifted"):
        r, p, u = ref[name]
        err = {"rho": r - r64, "p": p - p64, "u": (u - u64).norm(dim=0),
               "p_meanfree": (p - p.mean()) - (p64 - p64.mean())}
        e = {k: norms(v) for k, v in err.items()}
        ratio = {}
        for k in ("rho", "p", "u"):
            dk = out["discretisation"][k]
            src = e["p_meanfree"] if k == "p" else e[k]
            ratio[k] = {nn: src[nn] / dk[nn] for nn in ("L2", "Linf")}
        out["modes"][name] = {"error_vs_fp64": e, "ratio_to_discretisation_error": ratio}
    return out


def serve_run(rate, duration, budget, cell_cap, seed=4):
    """Poisson arrivals (rate per second for `duration` seconds) of D3Q19
    requests (edge log-uniform in [32, 192], 500-5000 steps, tau in
    [0.55, 1.0], seeded phi), FP32 shifted, served by the continuous-batching
    loop under an HBM budget.  Latency = arrival -> moments in host memory."""
    from paper_2208_09267_amd import serve
    from paper_2208_09267_amd import workloads as W

    arrivals = W.served_arrivals(rate=rate, duration=duration, seed=seed)
    offered = sum(w.ncells * w.steps for _, w in arrivals) / duration
    done = [0]

    def log(res):
        done[0] += 1
        if done[0] % 50 == 0:
            print("# served %d/%d (latency %.2f s)" % (done[0], len(arrivals), res.latency),
                  file=sys.stderr, flush=True)

    srv = serve.Server(budget_bytes=budget, cell_cap=cell_cap, log=log)
    t0 = time.perf_counter()
    results = srv.run(arrivals)
    wall = time.perf_counter() - t0
    out = serve.summarize(results, wall)
    lups = srv.stats["lups_two_step_tuning"] + srv.stats["lups_single_step_tuning"]
    stepping = lups / srv.time["step"] / 1e9 if srv.time["step"] > 0 else float("nan")
    out.update({"rate_per_s": rate, "arrival_window_s": duration,
                "offered_glups": offered / 1e9,
                # lattice updates per second while the batch steps: the capacity
                "stepping_glups": stepping, "offered_over_capacity": offered / 1e9 / stepping,
                "latency": "arrival -> moments (rho, p, u, FP64) copied into host memory",
                "hbm_budget_gb": budget / 1e9,
                "cell_cap": cell_cap, "batch_rebuilds": srv.stats["rebuilds"],
                "chunks": srv.stats["chunks"],
                "batch_steps_by_tuning": {"two_step": srv.stats["steps_two_step_tuning"],
                                          "single_step": srv.stats["steps_single_step_tuning"]},
                "lattice_updates_by_tuning": {"two_step": srv.stats["lups_two_step_tuning"],
                                              "single_step": srv.stats["lups_single_step_tuning"]},
                "loop_seconds": {k: round(v, 2) for k, v in srv.time.items()}})
    return out


def copy_probe(nbytes=1 << 30, reps=10):
    """Plain device-to-device copy through the library's copy kernel: the
    achievable streaming bandwidth (context for the roofline fraction) and
    the calibration kernel of the HBM traffic counters."""
    import torch

    from paper_2208_09267_amd import vanse

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    vanse.copy_probe(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        vanse.copy_probe(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert torch.equal(dst[:1024], src[:1024])
    return {"bytes_copied": nbytes, "ms": round(ms, 4),
            "gb_s": round(2 * nbytes / (ms / 1e3) / 1e9, 1),
            "frac_hbm": round(2 * nbytes / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}


def _cpu_model():
    """Host CPU model name (from /proc/cpuinfo) and logical core count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def _oracle_rate(w, pert, u0, seconds, threads, min_steps=2, max_steps=None):
    """Steps of workload w on the CPU oracle (FP64, as it stands) until
    `seconds` have passed (at least min_steps, at most max_steps): (MLUPS,
    steps, seconds)."""
    import oracle

    lat = {"D2Q9": oracle.D2Q9, "D3Q19": oracle.D3Q19}[w.lattice]
    eps0 = oracle.eps_at(w.dims, w.eps_mean, pert, w.period, 0)
    f = oracle.init(lat, w.dims, eps0, None, u0)
    steps, elapsed = 0, 0.0
    while (elapsed < seconds or steps < min_steps) and (max_steps is None or steps < max_steps):
        k = 1 if w.ncells > 100000 else 50
        if max_steps is not None:
            k = min(k, max_steps - steps)
        t0 = time.perf_counter()
        f, _ = oracle.run_separable(lat, w.dims, w.tau, w.eps_mean, pert, w.period, f, steps, k,
                                    quad_axes=w.quad_axes, fext=w.force, nthreads=threads)
        elapsed += time.perf_counter() - t0
        steps += k
    return w.ncells * steps / elapsed / 1e6, steps, elapsed


def cpu_baseline(w, pert, u0, seconds, full=False):
    """The CPU oracle (FP64, as it stands) on the host cores: the headline
    workload for a bounded number of steps on every core and on one core,
    the 64^2 D2Q9 workload in full (1000 steps) and a bounded sample of the
    128^3 workload (all of its 1000 steps with full=True)."""
    from paper_2208_09267_amd import workloads as W

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    model, ncpu = _cpu_model()
    rate, steps, el = _oracle_rate(w, pert, u0, seconds, threads)
    rate1, steps1, el1 = _oracle_rate(w, pert, u0, seconds / 3, 1, min_steps=1)
    w0 = W.d2q9_64()
    r0, s0, e0 = _oracle_rate(w0, w0.eps_pert(), None, 0.0, threads, max_steps=w0.steps,
                              min_steps=w0.steps)
    w1 = W.d3q19_128()
    if full:
        r1, s1, e1 = _oracle_rate(w1, w1.eps_pert(), w1.u0(), 0.0, threads,
                                  min_steps=w1.steps, max_steps=w1.steps)
    else:
        r1, s1, e1 = _oracle_rate(w1, w1.eps_pert(), w1.u0(), seconds / 3, threads)
    return {"value": rate, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d steps of the full %dx%dx%d D3Q19 FP64 workload (%.1f s)"
                      % (steps, w.dims[0], w.dims[1], w.dims[2], el),
            "host_cpu": model, "host_logical_cpus": ncpu,
            "one_thread": {"value": rate1, "unit": "MLUPS", "cores": 1,
                           "sample": "%d steps of the same workload (%.1f s)" % (steps1, el1)},
            "d2q9_64": {"value": r0, "unit": "MLUPS", "cores": threads,
                        "sample": "the full workload: %d steps of D2Q9 64^2 FP64 (%.2f s)"
                                  % (s0, e0)},
            "d3q19_128": {"value": r1, "unit": "MLUPS", "cores": threads,
                          "sample": "%d%s steps of D3Q19 128^3 FP64 (%.1f s)"
                                    % (s1, " (all)" if full else "", e1)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--variants", default="fp32_shifted,fp64,fp16_shifted,fx16_shifted",
                    help="comma list; the first one is the headline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time all 1000 steps of the 128^3 workload on the CPU oracle")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only the CPU oracle timings (no GPU)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched workloads and the served sample")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served samples (30 s of requests at 20/s, 15 s at 8/s)")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--no-d3q27", action="store_true")
    ap.add_argument("--no-single-step", action="store_true",
                    help="skip the single-step comparison run of two-step variants")
    ap.add_argument("--fixed-launch", action="store_true",
                    help="use the recorded launch shapes instead of autotuning")
    ap.add_argument("--fixed-shape", action="append", default=[],
                    help="with --fixed-launch: VARIANT=tile_x,tile_y,flat,rows,planes")
    ap.add_argument("--precision", action="store_true",
                    help="run the reduced-storage error study instead of the throughput bench")
    ap.add_argument("--serve", action="store_true",
                    help="run the served request stream instead of the throughput bench")
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--cell-cap", type=float, default=40e6)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2208_09267_amd import workloads as W

    if args.precision:
        torch.cuda.set_device(0)
        print(json.dumps({"precision": precision_study()}), flush=True)
        return
    if args.serve:
        torch.cuda.set_device(0)
        print(json.dumps({"served": serve_run(args.rate, args.duration, args.budget_gb * 1e9,
                                              int(args.cell_cap))}), flush=True)
        return

    w = W.d3q19_256()
    pert = w.eps_pert()
    u0 = w.u0()
    if args.cpu_only:
        print(json.dumps({"cpu_baseline": cpu_baseline(w, pert, u0, args.cpu_seconds,
                                                       args.cpu_full)}), flush=True)
        return
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pert_t = torch.from_numpy(pert).to(dev)
    u0_t = torch.from_numpy(np.ascontiguousarray(u0)).to(dev)

    for spec in args.fixed_shape:
        name, shape = spec.split("=")
        FIXED_LAUNCH[name] = tuple(int(v) for v in shape.split(","))
    variants = [v for v in args.variants.split(",") if v]
    results = {}
    for v in variants:
        results[v] = gpu_variant(v, w, pert_t, u0_t, args.steps, args.warmup, args.fixed_launch)
        print("# %s: %.1f MLUPS, %.4f ms/step, %s %.0f GB/s (%.1f%% of 8 TB/s; "
              "single-step equivalent %.1f%%)"
              % (v, results[v]["mlups"], results[v]["ms_per_step"], results[v]["kernel"],
                 results[v]["gb_s"], 100 * results[v]["frac_hbm"],
                 100 * results[v]["effective_frac"]), file=sys.stderr, flush=True)
    # the single-step kernel on the same workload, for comparison
    single = {}
    if not args.no_single_step:
        for v in variants:
            if results[v]["launch"]["two_step_rows"]:
                x = gpu_variant(v, w, pert_t, u0_t, min(args.steps, 400), args.warmup,
                                SINGLE_LAUNCH[v])
                single[v] = {"mlups": round(x["mlups"], 1), "ms_per_step": round(x["ms_per_step"], 5),
                             "gb_s": round(x["gb_s"], 1), "frac_hbm": round(x["frac_hbm"], 4),
                             "kernel": x["kernel"], "steps": x["steps"]}
                print("# %s single-step kernel: %.1f MLUPS" % (v, x["mlups"]), file=sys.stderr,
                      flush=True)

    head = variants[0]
    r = results[head]
    traffic = measured_traffic(head, r["kernel"])
    out = {
        "metric": METRIC,
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_NAME[head],
        "data": "synthetic",
        "config": {"workload": "D3Q19 VANSE-LBM 256^3 periodic, tau=0.55, seeded 8-mode Fourier "
                               "phi around 0.75 (seed 1, period 1000 steps), Taylor-Green u0 "
                               "amplitude 0.02",
                   "lattice": "D3Q19", "dims": list(w.dims), "tau": w.tau,
                   "storage": head, "global_batch": 1},
        "roofline": {"bound": "hbm", "kernel": r["kernel"],
                     "achieved": round(r["gb_s"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(r["frac_hbm"], 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "calibrated on a copy kernel)",
                     "algorithmic_bytes_per_launch": r["bytes_per_launch"],
                     "ms_per_launch": round(r["ms_per_launch"], 5),
                     "lups_per_launch": w.ncells * r["steps_per_launch"],
                     "bytes_per_lup": r["bytes_per_lup"],
                     "effective_gb_s_single_step_bytes": round(r["effective_gb_s"], 1),
                     "effective_frac_single_step_bytes": round(r["effective_frac"], 4),
                     "single_pass_bytes_per_lup": BYTES_PER_PASS[head],
                     "note": "achieved/frac: the kernel's own algorithmic bytes per launch "
                             "(populations read and written once, one phi value, per cell and "
                             "launch) over its HIP-event launch time; a two-step launch does two "
                             "lattice updates per cell for them.  effective_*_single_step_bytes "
                             "count single_pass_bytes_per_lup per lattice update, which assumes "
                             "one HBM pass per step: the bandwidth a one-step-per-pass kernel "
                             "would need for the same MLUPS (it can exceed the peak)."},
        "variants": {v: {"mlups": round(x["mlups"], 1), "ms_per_step": round(x["ms_per_step"], 5),
                         "kernel": x["kernel"], "ms_per_launch": round(x["ms_per_launch"], 5),
                         "gb_s": round(x["gb_s"], 1), "frac_hbm": round(x["frac_hbm"], 4),
                         "bytes_per_lup": x["bytes_per_lup"],
                         "effective_frac_single_step_bytes": round(x["effective_frac"], 4),
                         "launch": x["launch"]}
                     for v, x in results.items()},
    }
    if single:
        out["single_step_kernel"] = single
    if not args.no_copy_probe:
        out["copy_probe"] = copy_probe()
    if not args.no_d3q27:
        out["d3q27_256"] = d3q27_run()
        print("# d3q27: %s" % json.dumps(out["d3q27_256"]), file=sys.stderr, flush=True)
        out["small_configs"] = small_configs_run()
        print("# small configs: %s" % json.dumps(out["small_configs"]), file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = batched_run()
        print("# batched: %s" % json.dumps(out["batched"]), file=sys.stderr, flush=True)
        out["batched_256"] = batched_256_run()
        print("# batched 256^3: %s" % json.dumps(out["batched_256"]), file=sys.stderr, flush=True)
        if not args.no_serve:
            # the served workload's arrival rate (20 requests/s) over a 30 s
            # window of arrivals: offered load above capacity, so latency is
            # queueing; the 10-minute stream is `--serve --rate 20 --duration
            # 600`.  Then 8 requests/s (below capacity) for the latency of
            # the loop itself.
            out["served"] = serve_run(20.0, 30.0, args.budget_gb * 1e9, int(args.cell_cap))
            print("# served: %s" % json.dumps(out["served"]), file=sys.stderr, flush=True)
            out["served_below_capacity"] = serve_run(8.0, 15.0, args.budget_gb * 1e9,
                                                     int(args.cell_cap))
            print("# served below capacity: %s" % json.dumps(out["served_below_capacity"]),
                  file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, pert, u0, args.cpu_seconds, args.cpu_full)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
