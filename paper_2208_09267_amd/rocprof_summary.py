"""Summaries of rocprofv3 output for the measurement records.

CSV in, short text out: per-kernel launch statistics of a
``rocprofv3 --kernel-trace --stats`` run, and HBM bytes per dispatch of the
D3Q19 256^3 step kernels from two ``rocprofv3 --pmc`` runs (FETCH_SIZE, then
WRITE_SIZE) of ``bench.py --fixed-launch``, each counter scaled by what it
reads for the library's copy kernel moving a known number of bytes in the same
run.

Usage (repository root):
  python -m paper_2208_09267_amd.rocprof_summary stats DIR
  python -m paper_2208_09267_amd.rocprof_summary trace DIR
  python -m paper_2208_09267_amd.rocprof_summary sq DIR [DIR ...]
  python -m paper_2208_09267_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR [FETCH_DIR WRITE_DIR ...] OUT_JSON
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
NCELLS_256 = 256 ** 3
COPY_BYTES = 1 << 30            # bytes copied by bench.py's copy_probe
MODES = {0: "fp64", 1: "fp32_shifted", 2: "fp16_shifted", 3: "fx16_shifted"}
MODE_LABEL = {0: "FP64", 1: "FP32_SHIFTED", 2: "FP16_SHIFTED", 3: "FX16_SHIFTED"}
ELEM = {0: 8, 1: 4, 2: 2, 3: 2}
PERT = {0: 8, 1: 4, 2: 4, 3: 4}
LATTICE_Q = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}


def kernel_source_hash() -> str:
    """Hash of the sources that define the step kernels (a traffic record is
    valid only for the kernels it was measured on)."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "lattice.h", "internal.h"):
        with open(os.path.join(HERE, "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_label(kind: str, lattice: str, mode: int, rows=None) -> str:
    """'step_kernel<D3Q19, FP32_SHIFTED>' or, for the two-step kernel with
    tile rows, 'fused2_kernel<D3Q19, FP32_SHIFTED, rows 4>'."""
    if kind == "fused2_kernel" and rows:
        return "%s<%s, %s, rows %d>" % (kind, lattice, MODE_LABEL[mode], rows)
    return "%s<%s, %s>" % (kind, lattice, MODE_LABEL[mode])


def parse_name(full: str):
    """(label, lattice, mode) of a step kernel's demangled rocprofv3 name, or
    None for other kernels.  The two-step kernel's label carries its tile
    rows when they are a compile-time argument."""
    m = re.search(r"vanse::(fused2_kernel|step_kernel)<vanse::(D\dQ\d+), (\d)((?:, \w+)*)>", full)
    if not m:
        return None
    kind, lat, mode = m.group(1), m.group(2), int(m.group(3))
    rows = None
    if kind == "fused2_kernel":
        args = [a.strip() for a in m.group(4).split(",") if a.strip()]
        if len(args) >= 4 and args[3].isdigit() and int(args[3]) > 0:
            rows = int(args[3])
    return kernel_label(kind, lat, mode, rows), lat, mode


def _one(pattern):
    files = sorted(glob.glob(pattern))
    if not files:
        raise FileNotFoundError(pattern)
    return files[0]


def _counters(directory):
    """{full kernel name: [counter value per dispatch]} (KiB)."""
    out = {}
    with open(_one(os.path.join(directory, "*counter_collection.csv"))) as fh:
        for row in csv.DictReader(fh):
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def traffic(pairs):
    """pairs: [(FETCH_SIZE run dir, WRITE_SIZE run dir), ...] of the same
    kernels; each run is calibrated on its own copy kernel."""

    def calib(rows, name):
        vals = [v for k, vs in rows.items() if "copy_kernel" in k for v in vs]
        if not vals:
            raise RuntimeError("no copy_kernel dispatch in the %s run" % name)
        kib = sum(vals) / len(vals)
        return kib, COPY_BYTES / (kib * 1024.0)

    kernels = {}
    calibration = []
    for fetch_dir, write_dir in pairs:
        fetch, write = _counters(fetch_dir), _counters(write_dir)
        f_kib, f_scale = calib(fetch, "FETCH_SIZE")
        w_kib, w_scale = calib(write, "WRITE_SIZE")
        calibration.append({"copy_kernel_bytes": COPY_BYTES, "FETCH_SIZE_KiB": f_kib,
                            "WRITE_SIZE_KiB": w_kib, "fetch_scale": f_scale,
                            "write_scale": w_scale})
        for full in sorted(set(fetch) & set(write)):
            p = parse_name(full)
            if p is None:
                continue
            label, lat, mode = p
            fb = sum(fetch[full]) / len(fetch[full]) * 1024.0 * f_scale
            wb = sum(write[full]) / len(write[full]) * 1024.0 * w_scale
            k = kernels.setdefault(label, {"rocprof_names": [], "dispatches": 0, "fetch_bytes": [],
                                           "write_bytes": [], "mode": mode, "lattice": lat})
            if full not in k["rocprof_names"]:
                k["rocprof_names"].append(full)
            k["dispatches"] += len(fetch[full])
            k["fetch_bytes"].append(fb)
            k["write_bytes"].append(wb)
    for label, k in kernels.items():
        q = LATTICE_Q[k["lattice"]]
        mode = k["mode"]
        k["fetch_bytes"] = sum(k["fetch_bytes"]) / len(k["fetch_bytes"])  # mean over parities/runs
        k["write_bytes"] = sum(k["write_bytes"]) / len(k["write_bytes"])
        k["bytes_per_launch"] = k["fetch_bytes"] + k["write_bytes"]
        alg_read = (q * ELEM[mode] + PERT[mode]) * NCELLS_256
        alg_write = q * ELEM[mode] * NCELLS_256
        k["algorithmic_read_bytes"] = alg_read
        k["algorithmic_write_bytes"] = alg_write
        k["algorithmic_bytes_per_launch"] = alg_read + alg_write
        k["fetch_ratio"] = k["fetch_bytes"] / alg_read
        k["write_ratio"] = k["write_bytes"] / alg_write
        k["ratio_to_algorithmic"] = k["bytes_per_launch"] / (alg_read + alg_write)
    return {
        "kernel_source_hash": kernel_source_hash(),
        "workload": "D3Q19 256^3 (bench.py --fixed-launch)",
        "calibration": calibration,
        "kernels": kernels,
    }


def stats(directory):
    """Rows of (kernel, calls, average us, min us, max us) for vanse kernels."""
    rows = []
    with open(_one(os.path.join(directory, "*kernel_stats.csv"))) as fh:
        for row in csv.DictReader(fh):
            name = row["Name"]
            if "vanse::" not in name:
                continue
            short = re.sub(r"\(.*\)$", "", name).replace("void ", "").replace("vanse::", "")
            rows.append((short, int(row["Calls"]), float(row["AverageNs"]) / 1e3,
                         float(row["MinNs"]) / 1e3, float(row["MaxNs"]) / 1e3))
    return rows


# cells of the bench.py workloads a kernel launch of the kernel trace belongs to
_BATCH64_CELLS = 22179840        # the 64-solve batch
_BATCH256_CELLS = 4 * 256 ** 3   # four 256^3 solves


def _workload(short, grid):
    """(workload name, cells) of a launch in a bench.py run, from the kernel
    name and its grid size; (None, None) for other kernels."""
    lat = "D2Q9" if "D2Q9" in short else ("D3Q27" if "D3Q27" in short else "D3Q19")
    if short.startswith("batch_fused2"):
        if ", 256, 4" in short:
            return "4 x 256^3 batch", _BATCH256_CELLS
        return "64-solve batch", _BATCH64_CELLS
    if short.startswith("batch_step"):
        if grid >= _BATCH256_CELLS - 1024:
            return "4 x 256^3 batch", _BATCH256_CELLS
        return "64-solve batch", _BATCH64_CELLS
    if lat == "D2Q9" and short.startswith("step_kernel"):
        return "D2Q9 64^2", 64 * 64
    if short.startswith("fused2"):
        return ("D3Q19 128^3", 128 ** 3) if ", 128, 4" in short else (lat + " 256^3", 256 ** 3)
    if short.startswith("step_kernel"):
        return ("D3Q19 128^3", 128 ** 3) if grid < 4000000 else (lat + " 256^3", 256 ** 3)
    return None, None


def trace(directory, min_calls=50):
    """Rows of (kernel, workload, calls, average us, min us, max us,
    algorithmic GB/s, MLUPS) from a --kernel-trace run of bench.py, grouped by
    kernel and grid size (groups with fewer calls are autotuner trials)."""
    groups = {}
    with open(_one(os.path.join(directory, "*kernel_trace.csv"))) as fh:
        for row in csv.DictReader(fh):
            name = row["Kernel_Name"]
            if "vanse::" not in name:
                continue
            short = re.sub(r"\(.*\)$", "", name).replace("void ", "").replace("vanse::", "")
            us = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3
            groups.setdefault((short, int(row["Grid_Size_X"])), []).append(us)
    rows = []
    for (short, grid), d in groups.items():
        if len(d) < min_calls:
            continue
        avg = sum(d) / len(d)
        wl, cells = _workload(short, grid)
        m = re.match(r"(\w+)<(D\dQ\d+), (\d)", short)
        gbs = mlups = None
        if wl is not None and m:
            q = LATTICE_Q[m.group(2)]
            mode = int(m.group(3))
            lups = (2 if "fused2" in short else 1) * cells
            gbs = (2 * q * ELEM[mode] + PERT[mode]) * cells / (avg * 1e-6) / 1e9
            mlups = lups / (avg * 1e-6) / 1e6
        rows.append((short, wl, len(d), avg, min(d), max(d), gbs, mlups))
    return sorted(rows, key=lambda r: (r[1] or "~", r[0]))


def sq(directories):
    """Per-kernel mean of every SQ counter in the given --pmc runs (one
    counter group per run), for the step kernels; with the derived shares of
    a wave's lifetime spent issuing VALU instructions, issuing anything, and
    waiting on a memory or LDS result (the SQ_*_CYCLES-type counters are
    in the same units, so their ratios are unit-free)."""
    per = {}
    for d in directories:
        with open(_one(os.path.join(d, "*counter_collection.csv"))) as fh:
            for row in csv.DictReader(fh):
                p = parse_name(row["Kernel_Name"])
                if p is None:
                    continue
                per.setdefault(p[0], {}).setdefault(row["Counter_Name"], []).append(
                    float(row["Counter_Value"]))
    out = {}
    for label, cs in per.items():
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        wc = m.get("SQ_WAVE_CYCLES")
        if wc:
            for c, share in (("SQ_ACTIVE_INST_VALU", "valu_share"),
                             ("SQ_ACTIVE_INST_ANY", "issue_share"),
                             ("SQ_WAIT_INST_ANY", "wait_share"),
                             ("SQ_ACTIVE_INST_SCA", "salu_share"),
                             ("SQ_ACTIVE_INST_LDS", "lds_share")):
                if c in m:
                    m[share] = m[c] / wc
        if "SQ_WAVES" in m and wc:
            m["wave_cycles_per_wave"] = wc / m["SQ_WAVES"]
        out[label] = m
    return out


def main(argv):
    if len(argv) >= 2 and argv[0] == "sq":
        for label, m in sorted(sq(argv[1:]).items()):
            print(label)
            for k in sorted(m):
                print("  %-28s %.4g" % (k, m[k]))
        return 0
    if len(argv) >= 2 and argv[0] == "trace":
        for k, wl, n, avg, mn, mx, gbs, mlups in trace(argv[1]):
            launch_bound = wl == "D2Q9 64^2"
            print("| `%s` | %s | %d | %.1f | %.1f | %.1f | %s | %s |"
                  % (k, wl or "—", n, avg, mn, mx,
                     "—" if gbs is None or launch_bound else "%.0f" % gbs,
                     "—" if mlups is None else ("%.0f" % mlups) +
                     (" (launch-bound)" if launch_bound else "")))
        return 0
    if len(argv) >= 2 and argv[0] == "stats":
        for r in stats(argv[1]):
            print("| `%s` | %d | %.1f | %.1f | %.1f |" % r)
        return 0
    if len(argv) >= 4 and len(argv) % 2 == 0 and argv[0] == "traffic":
        rec = traffic(list(zip(argv[1:-1:2], argv[2:-1:2])))
        with open(argv[-1], "w") as fh:
            json.dump(rec, fh, indent=1)
        for label, k in sorted(rec["kernels"].items()):
            print("%-40s fetch %.4g B (%.3f x)  write %.4g B (%.3f x)  per launch %.4g B (%.3f x)"
                  % (label, k["fetch_bytes"], k["fetch_ratio"], k["write_bytes"],
                     k["write_ratio"], k["bytes_per_launch"], k["ratio_to_algorithmic"]))
        return 0
    print(__doc__, file=sys.stderr)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
