"""Host logic of bench.py (no GPU): kernel tags from demangled names, algorithmic bytes per lattice
update, and the rocprofv3 summary with its counter calibration on the 1 GiB copy."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2206_02145_amd import workloads as W  # noqa: E402

FLOW32 = "void lbcg::step_single<3, true, float, float, 64, 2, 4, false, 2, 0, false, false>(lbcg::InstDev, int)"
FLOW16 = "void lbcg::step_single<3, true, float, __half, 64, 2, 4, false, 2, 0, false, false>(lbcg::InstDev, int)"
CHM = "void lbcg::step_single<3, true, float, float, 64, 2, 4, false, 2, 0, false, true>(lbcg::InstDev, int)"
WALLS = "void lbcg::step_single<3, true, float, float, 64, 2, 4, false, 2, 0, true, false>(lbcg::InstDev, int)"
NOFLOW = "void lbcg::step_single<3, false, float, float, 64, 2, 4, false, 0, 0, false, false>(lbcg::InstDev, int)"
BATCH = "void lbcg::step_batch<2, true, float, float, 64, 4, 1, false, 2, 0, false>(lbcg::InstDev const*, int, int)"


def test_kernel_tags():
    assert bench._kernel_tag(FLOW32) == "step_3d_flow_fp32"
    assert bench._kernel_tag(FLOW16) == "step_3d_flow_fp16shift"
    assert bench._kernel_tag(CHM) == "step_3d_flow_chmrt_fp32"
    assert bench._kernel_tag(WALLS) == "step_3d_flow_walls_fp32"
    assert bench._kernel_tag(NOFLOW) == "step_3d_noflow_fp32"
    assert bench._kernel_tag(BATCH) == "step_batch_2d_flow_fp32"
    assert bench._kernel_tag("void lbcg::mlp::gemm_bf16<3>(lbcg::mlp::GemmArgs)") == "gemm_bf16_dw"
    assert bench._kernel_tag("lbcg::mlp::adam_kernel(long long, float*)") == "adam_kernel"
    assert bench._kernel_tag("__amd_rocclr_copyBuffer") == "copy_1GiB"


def test_bytes_per_lattice_update():
    """Every population read and written once, plus phi_prev: 3-D flow binary32 2 (2*7*4 + 19*4 +
    4) = 272 B, binary16 flow storage 196 B, 3-D without flow 120 B, 2-D flow 160 B."""
    assert bench.bytes_per_lup(W.config3(), "fp32") == 272
    assert bench.bytes_per_lup(W.config3(), "fp16shift") == 196
    assert bench.bytes_per_lup(W.config2(), "fp32") == 120
    assert bench.bytes_per_lup(W.sweep_instance(64, 0.1, 5.0, 0.01), "fp32") == 160
    assert bench.bytes_per_lup(W.params(dim=2, nx=8, ny=8), "fp64") == 2 * (2 * 5 * 8 + 8)


def write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_summary_calibrates_on_the_large_copy(tmp_path):
    """Synthetic rocprofv3 output: five 1 GiB copies among small runtime copies, and a step kernel.
    The calibration uses only the large copies; the kernel's bytes are scaled by it."""
    d = str(tmp_path / "run")
    trace = []
    t = 0
    for name, us in [("__amd_rocclr_copyBuffer", 2.0)] * 7 + [("__amd_rocclr_copyBuffer", 400.0)] * 5 + \
            [(FLOW32, 186.0)] * 4:
        trace.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + int(us * 1000)})
        t += 10 ** 6
    write_csv(f"{d}/prof_kt/run_kernel_trace.csv", trace)
    gib_kib = (1 << 30) / 1024
    for sub, cname, scale in (("prof_fetch", "FETCH_SIZE", 0.5), ("prof_write", "WRITE_SIZE", 1.0)):
        rows = [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": cname, "Counter_Value": 3.0}] * 7
        rows += [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": cname, "Counter_Value": gib_kib * scale}] * 5
        # the step kernel: 474.5 MB read, 438.3 MB written, counted at the same scale
        true = 474.5e6 if cname == "FETCH_SIZE" else 438.3e6
        rows += [{"Kernel_Name": FLOW32, "Counter_Name": cname, "Counter_Value": true / 1024 * scale}] * 4
        write_csv(f"{d}/{sub}/run_counter_collection.csv", rows)
    out = str(tmp_path / "profiles")
    bench.summarize_profiles(d, out)
    with open(os.path.join(out, "traffic.json")) as fh:
        tr = json.load(fh)
    e = tr["step_3d_flow_fp32"]
    assert e["read_bytes"] == pytest.approx(474.5e6, rel=1e-9)
    assert e["write_bytes"] == pytest.approx(438.3e6, rel=1e-9)
    assert e["avg_us"] == pytest.approx(186.0)
    assert e["kernel_source_hash"] == bench.kernel_source_hash()
    md = open(os.path.join(out, "step_3d_flow_c3.md")).read()
    assert "FETCH_SIZE x 2.000, WRITE_SIZE x 1.000" in md
    assert "| copy_1GiB | 5 | 400.0 |" in md
    assert "| 855.6 | 1.067 |" in md
