"""CPU tests of bench.py's host side: the one-GPU guard, the kernel labels
that key the committed counter record, and the record's use as
roofline.traffic (only while the kernel source matches the hash it was
measured on)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2208_09267_amd import rocprof_summary as rs  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("full,label", [
    ("void vanse::fused2_kernel<vanse::D3Q19, 1, 1, 2, 256, 4, false, 1024>(vanse::StepArgs)",
     "fused2_kernel<D3Q19, FP32_SHIFTED, rows 4>"),
    ("void vanse::fused2_kernel<vanse::D3Q19, 0, 1, 2, 256, 2, false, 512>(vanse::StepArgs)",
     "fused2_kernel<D3Q19, FP64, rows 2>"),
    ("void vanse::step_kernel<vanse::D3Q19, 2, 1, true, 0>(vanse::StepArgs)",
     "step_kernel<D3Q19, FP16_SHIFTED>"),
    ("void vanse::fused2_kernel<vanse::D3Q19, 3, 1, 2, 256, 4, false, 1024>(vanse::StepArgs)",
     "fused2_kernel<D3Q19, FX16_SHIFTED, rows 4>"),
])
def test_rocprof_names_map_to_bench_labels(full, label):
    assert rs.parse_name(full)[0] == label
    variant = {0: "fp64", 1: "fp32_shifted", 2: "fp16_shifted",
               3: "fx16_shifted"}[rs.parse_name(full)[2]]
    rows = 4 if "rows 4" in label else (2 if "rows 2" in label else 0)
    assert bench.kernel_name(variant, rows) == label


def test_traffic_record_used_only_for_the_kernel_source_it_measured(tmp_path, monkeypatch):
    path = os.path.join(ROOT, "profiles", "traffic_d3q19_256.json")
    rec = json.load(open(path))
    label = bench.kernel_name("fp32_shifted", 4)
    if rec["kernel_source_hash"] == rs.kernel_source_hash():
        assert bench.measured_traffic("fp32_shifted", label) == \
            round(rec["kernels"][label]["bytes_per_launch"])
    # a record taken on other kernel sources is not used
    stale = dict(rec, kernel_source_hash="0" * 16)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_d3q19_256.json").write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("fp32_shifted", label) is None
