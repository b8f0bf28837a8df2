#!/usr/bin/env python3
"""Throughput of the fused VANSE lattice Boltzmann step on one MI355X.

Workload (the headline configuration): D3Q19, 256^3 periodic, tau = 0.55,
phi(x, t_n) = 0.75 + cos(2 pi n / 1000) * dphi(x) with dphi the seeded sum of
8 Fourier modes (seed 1), Taylor-Green initial velocity of amplitude 0.02,
rho = 1.  Storage variants: FP32 shifted populations (headline), FP64 and
FP16 shifted.  One "step" is one full time step of the whole lattice; the
state is resident in HBM before timing starts.

Prints ONE JSON line (rank 0).  `value` is the headline variant's MLUPS;
`roofline` describes its step kernel against the 8 TB/s HBM peak using
algorithmic bytes per lattice update (Q loads + Q stores + one phi value);
`cpu_baseline` times the FP64 CPU oracle on a bounded number of steps of the
same workload on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline, D3Q19 256³ FP64 vs FP32-shifted; p50/p99 solve latency"
PEAK_HBM_GBS = 8000.0
# algorithmic bytes per lattice update: Q loads + Q stores + one phi value
BYTES_PER_LUP = {"fp64": 19 * 8 * 2 + 8, "fp32_shifted": 19 * 4 * 2 + 4,
                 "fp16_shifted": 19 * 2 * 2 + 4}
DTYPE_NAME = {"fp64": "f64", "fp32_shifted": "f32", "fp16_shifted": "f32"}
KERNEL_NAME = {"fp64": "step_kernel<D3Q19, FP64>",
               "fp32_shifted": "step_kernel<D3Q19, FP32_SHIFTED>",
               "fp16_shifted": "step_kernel<D3Q19, FP16_SHIFTED>"}


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("kernels.hip", "lattice.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2208_09267_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(variant):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_d3q19_256.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = rec.get("variants", {}).get(variant)
    return None if v is None else v.get("bytes_per_launch")


def gpu_variant(variant, w, pert_t, u0_t, steps, warmup):
    import torch

    from paper_2208_09267_amd import vanse

    s = vanse.Solver(w.lattice, w.dims, w.tau, vanse.DTYPES[variant])
    s.set_porosity(w.eps_mean, pert_t, w.period, w.quad_axes)
    s.set_force(w.force)
    s.init(None, u0_t)
    s.step(warmup)
    torch.cuda.synchronize()
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
    mlups = w.ncells * steps / (ms / 1e3) / 1e6
    gbs = BYTES_PER_LUP[variant] * w.ncells / (ms_step / 1e3) / 1e9
    return {"mlups": mlups, "ms_per_step": ms_step, "wall_s": wall, "gb_s": gbs,
            "frac_hbm": gbs / PEAK_HBM_GBS, "bytes_per_lup": BYTES_PER_LUP[variant],
            "mass": mass}


def cpu_baseline(w, pert, u0, seconds):
    """The CPU oracle (FP64, as it stands) on the same workload, timed for a
    bounded number of steps."""
    import oracle

    lat = oracle.D3Q19
    eps0 = oracle.eps_at(w.dims, w.eps_mean, pert, w.period, 0)
    f = oracle.init(lat, w.dims, eps0, None, u0)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    steps, elapsed = 0, 0.0
    while elapsed < seconds or steps < 2:
        t0 = time.perf_counter()
        f, _ = oracle.run_separable(lat, w.dims, w.tau, w.eps_mean, pert, w.period, f, steps, 1,
                                    fext=w.force, nthreads=threads)
        elapsed += time.perf_counter() - t0
        steps += 1
    return {"value": w.ncells * steps / elapsed / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d steps of the full %dx%dx%d D3Q19 FP64 workload (%.1f s)"
                      % (steps, w.dims[0], w.dims[1], w.dims[2], elapsed)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--variants", default="fp32_shifted,fp64,fp16_shifted",
                    help="comma list; the first one is the headline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2208_09267_amd import workloads as W

    w = W.d3q19_256()
    pert = w.eps_pert()
    u0 = w.u0()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pert_t = torch.from_numpy(pert).to(dev)
    u0_t = torch.from_numpy(np.ascontiguousarray(u0)).to(dev)

    variants = [v for v in args.variants.split(",") if v]
    results = {}
    for v in variants:
        results[v] = gpu_variant(v, w, pert_t, u0_t, args.steps, args.warmup)
        print("# %s: %.1f MLUPS, %.4f ms/step, %.0f GB/s (%.1f%% of 8 TB/s)"
              % (v, results[v]["mlups"], results[v]["ms_per_step"], results[v]["gb_s"],
                 100 * results[v]["frac_hbm"]), file=sys.stderr, flush=True)

    head = variants[0]
    r = results[head]
    traffic = measured_traffic(head)
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
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAME[head],
                     "achieved": round(r["gb_s"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(r["frac_hbm"], 4), "traffic": traffic,
                     "bytes_per_lup": r["bytes_per_lup"], "lups_per_launch": w.ncells},
        "variants": {v: {"mlups": round(x["mlups"], 1), "ms_per_step": round(x["ms_per_step"], 5),
                         "gb_s": round(x["gb_s"], 1), "frac_hbm": round(x["frac_hbm"], 4),
                         "bytes_per_lup": x["bytes_per_lup"]} for v, x in results.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, pert, u0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
