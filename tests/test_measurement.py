"""Host logic of the measurement: the profile summariser (rocprof_summary) on synthetic
rocprofv3 output, and the bench's per-iteration byte counts.

The summariser scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what the same counters
read for a plain copy of 1 GiB, averages over dispatches, joins the counter rows (rocprof
kernel names) with the bench's HIP-event timing names and writes the per-launch HBM bytes
that bench.py reports as roofline.traffic."""
import csv
import json
import os

import pytest

import bench
from paper_1612_06424_amd import rocprof_summary as rs


def test_timing_names_of_kernel_instances():
    assert rs.timing_name("k_dslash<double, 0, 0, 256, 2, true>") == "k_dslash<double, 0, 0, 256, 2>"
    assert rs.timing_name("k_dslash<float, 1, 3, 128, 1, false>") == "k_dslash<float, 1, 3, 128>"
    assert rs.timing_name("k_dslash<double, 0, 0, 128>") == "k_dslash<double, 0, 0, 128>"
    eo = "k_eo_hop_nt<float, 1, 4, 256, true, 2, true>"
    assert rs.timing_name(eo) == eo
    assert rs.short_name("void dd::(anonymous namespace)::k_eo_hop_nt<float, 1, 4, 256, true, 2, true>"
                         "(dd::Geo, dd::cpx<float> const*)") == eo


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summary_scales_counters_by_the_copy_and_joins_timing_names(tmp_path):
    d = tmp_path
    copy = "__amd_rocclr_copyBuffer"
    hop = "k_eo_hop_nt<float, 1, 4, 256, true, 2, true>"
    dsl = "k_dslash<double, 0, 0, 256, 2, true>"
    # the plain 1 GiB copy reads half its bytes in FETCH_SIZE (x2) and all of them in WRITE_SIZE
    _counter_csv(d / "copy_fetch", [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="FETCH_SIZE",
                                         Counter_Value=(1 << 30) / 2 / 1024)])
    _counter_csv(d / "copy_write", [dict(Dispatch_Id=1, Kernel_Name=copy, Counter_Name="WRITE_SIZE",
                                         Counter_Value=(1 << 30) / 1024)])
    # two dispatches of each kernel: the summary averages them
    _counter_csv(d / "fetch", [dict(Dispatch_Id=i, Kernel_Name=k, Counter_Name="FETCH_SIZE", Counter_Value=v)
                               for i, k, v in ((3, hop, 1000.0), (4, hop, 3000.0), (5, dsl, 500.0), (6, dsl, 500.0))])
    _counter_csv(d / "write", [dict(Dispatch_Id=i, Kernel_Name=k, Counter_Name="WRITE_SIZE", Counter_Value=v)
                               for i, k, v in ((3, hop, 100.0), (4, hop, 300.0), (5, dsl, 50.0), (6, dsl, 50.0))])
    os.makedirs(d / "trace", exist_ok=True)
    with open(d / "trace" / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow(dict(Name=hop, Calls=2, TotalDurationNs=800000, AverageNs=400000, Percentage=80.0))
        w.writerow(dict(Name=dsl, Calls=2, TotalDurationNs=200000, AverageNs=100000, Percentage=20.0))
    # the bench line of the traced run: HIP-event timing by the library's names
    kt = {hop: {"ms": 0.8, "launches": 2, "GBs": 4000.0}, "k_dslash<double, 0, 0, 256, 2>": {"ms": 0.2, "launches": 2,
                                                                                              "GBs": 5000.0}}
    line = {"metric": "m", "value": 1.0, "roofline": {"kernel": hop}, "stencil_kernels": kt}
    (d / "trace.log").write_text("[bench] x\n" + json.dumps(line) + "\n")
    rs.main([str(d)])
    rec = json.load(open(d / "stencil_traffic.json"))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["source_hash"] == rs.kernel_source_hash()
    h = rec["kernels"][hop]
    assert h["launches"] == 2
    assert h["fetch_bytes"] == round(2000.0 * 1024 * 2) and h["write_bytes"] == round(200.0 * 1024)
    assert h["hbm_bytes"] == h["fetch_bytes"] + h["write_bytes"]
    assert h["algorithmic_bytes"] == round(4000.0 * 0.8 * 1e6 / 2)
    # the full stencil's counter rows carry the lane-permute flag, its timing name does not
    assert rec["kernels"]["k_dslash<double, 0, 0, 256, 2>"]["algorithmic_bytes"] == round(5000.0 * 0.2 * 1e6 / 2)
    text = open(d / "summary.md").read()
    assert "Stencil source hash" in text and hop in text
    assert not list((d / "fetch").glob("*.csv"))  # raw files removed unless --keep-raw


@pytest.mark.parametrize("method,per_col", [("cgnr", 432), ("bicgstab", 624)])
@pytest.mark.parametrize("prec,rb,links", [("mixed", 4, 96), ("fp64", 8, 144)])
def test_iteration_bytes(method, per_col, prec, rb, links):
    nh, ncol = 1000, 12
    assert bench.eo_iteration_bytes(nh, ncol, prec, method) == nh * (per_col * ncol + 4 * links) * rb
