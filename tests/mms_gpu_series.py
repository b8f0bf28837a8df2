"""Convergence series of the travelling manufactured solutions on the GPU
(FP64), beyond what the CPU oracle reaches: errors of velocity and mean-free
pressure (physical units; L1, L2, Linf) once stabilised, and the order
between consecutive resolutions.  Same driver as tests/test_gpu_mms.py.

Usage (one MI355X): python tests/mms_gpu_series.py OUT.json EX:N1,N2,...:T_END ...
e.g. python tests/mms_gpu_series.py mms.json 4:36,48,72,96:10 5:24,32,48,64:8
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import mms_inputs as MI  # noqa: E402
from test_gpu_mms import gpu_mms  # noqa: E402


def series(ex, Ns, t_end, tau=0.5075, period_s=4.0):
    """Errors at t_end, and the change from t_end - period_s (the same phase
    of the travelling fields, which repeat every 4 s)."""
    out = {"example": ex, "tau": tau, "t_end_s": t_end, "runs": []}
    prev = None
    for N in Ns:
        dt = MI.setup(ex, N, tau)[5]
        nsteps = int(round(t_end / dt))
        samples = [max(1, nsteps - int(round(period_s / dt))), nsteps]
        t0 = time.perf_counter()
        errs, _ = gpu_mms(ex, N, tau, nsteps, samples=samples, progress=True)
        wall = time.perf_counter() - t0
        last, before = errs[samples[-1]], errs[samples[-2]]
        run = {"N": N, "steps": nsteps, "wall_s": round(wall, 1),
               "us_per_step": round(1e6 * wall / nsteps, 1),
               "errors_u_L1_L2_Linf_p_L1_L2_Linf": [float(v) for v in last],
               "relative_change_last_two_samples": [float(v) for v in np.abs(last - before) / last]}
        if prev is not None:
            run["order_from_previous"] = [float(v) for v in
                                          np.log(prev[1] / last) / np.log(N / prev[0])]
        prev = (N, last)
        out["runs"].append(run)
        print(json.dumps(run), flush=True)
    return out


if __name__ == "__main__":
    path = sys.argv[1]
    res = []
    for spec in sys.argv[2:]:
        ex, ns, t_end = spec.split(":")
        res.append(series(int(ex), [int(v) for v in ns.split(",")], float(t_end)))
        with open(path, "w") as fh:
            json.dump({"mms_gpu_series": res}, fh, indent=1)
