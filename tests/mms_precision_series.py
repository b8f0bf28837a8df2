"""Example 1 of the numerical validation (stationary, 2-D, D2Q9) on the GPU
in every storage mode, N = 32, 64, 128 (tau = 0.53, diffusive scaling,
errors at 16 s): how far each mode keeps the second order of the FP64 path.
Same driver as tests/test_gpu_next.py.

Usage (one MI355X): python tests/mms_precision_series.py OUT.json
"""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2208_09267_amd import vanse  # noqa: E402
from test_gpu_next import _gpu_mms  # noqa: E402

MODES = [("fp64", vanse.FP64), ("fp32_shifted", vanse.FP32_SHIFTED),
         ("fx16_shifted", vanse.FX16_SHIFTED), ("fp16_shifted", vanse.FP16_SHIFTED)]

if __name__ == "__main__":
    Ns = (32, 64, 128)
    out = {"example": 1, "tau": 0.53, "t_end_s": 16.0, "N": list(Ns), "modes": {}}
    for name, dt in MODES:
        e = np.array([_gpu_mms(1, N, 0.53, 16.0, dtype=dt, stabilised=False) for N in Ns])
        out["modes"][name] = {
            "errors_u_L1_L2_Linf_p_L1_L2_Linf": e.tolist(),
            "order": [np.round(np.log2(e[k] / e[k + 1]), 3).tolist() for k in range(len(Ns) - 1)]}
        print(json.dumps({name: out["modes"][name]}), flush=True)
        with open(sys.argv[1], "w") as fh:
            json.dump({"mms_precision_series": out}, fh, indent=1)
