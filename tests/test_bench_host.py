"""Host logic of bench.py, on the CPU: the roofline object of the JSON line,
the kernel names the profile summaries are keyed by, the grouping of counter
dispatches, and the refusal of more than one GPU."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def fake_run(variant, tuning, kernel_us=250.0, n=4096):
    cells = n * n
    K = max(1, tuning.get("fused_steps", 1))
    gbs = bench.BYTES_PER_CELL[variant] * cells / (kernel_us * 1e-6) / 1e9
    return {"tuning": tuning, "fused_steps": K, "rows": tuning.get("rows_per_strip", 0), "cells": cells,
            "kernel_avg_us": kernel_us, "achieved_GBs": gbs, "effective_GBs": K * gbs,
            "achieved_TFLOPs": bench.FLOPS_PER_CELL * K * cells / (kernel_us * 1e-6) / 1e12}


@pytest.mark.parametrize("variant", ["f64", "f32c", "f32"])
def test_roofline_object_has_the_contract_keys(variant):
    """Every precision's roofline is placed against HBM: algorithmic bytes of a
    launch over its duration, against 8 TB/s; the fused launch's vector
    figures ride along under their own keys."""
    shape = dict(zip(("rows_per_strip", "threads", "fused_steps", "lane_shift"), bench.HEADLINE_SHAPE[variant]))
    for tuning in (shape, {"fused_steps": 1, "threads": 0, "lane_shift": 0}):
        r = fake_run(variant, tuning)
        roof = bench.roofline_of(variant, r)
        for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
            assert key in roof
        assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == bench.PEAK_HBM_GBS
        assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"])
        assert roof["achieved"] == pytest.approx(bench.BYTES_PER_CELL[variant] * r["cells"] / 250e-6 / 1e9)
        if tuning is shape:
            assert roof["valu_frac"] == pytest.approx(roof["valu_TFLOPs"] / bench.PEAK_VALU_TFLOPS)
            if "valu_issue_frac" in roof:
                assert 0.0 < roof["valu_issue_frac"] <= 1.0
        if roof["traffic"] is not None:
            assert roof["hbm_measured_GBs"] == pytest.approx(roof["traffic"] / (250e-6) / 1e9)
        else:
            assert "hbm_measured_GBs" not in roof


def test_host_identity_names_the_cpu():
    h = bench.host_identity()
    assert h["nproc"] >= 1 and h["usable_cpus"] >= 1


def test_headline_kernel_names():
    names = {v: bench.kernel_name(v, dict(zip(("rows_per_strip", "threads", "fused_steps", "lane_shift"),
                                               bench.HEADLINE_SHAPE[v]))) for v in bench.HEADLINE_SHAPE}
    assert names["f64"] == ("fused_dpp_kernel<double, false, 2, 4>", "wide4")
    assert names["f32c"] == ("fused_dpp_kernel<float, true, 2, 4>", "lanes4")
    assert names["f32"] == ("fused_dpp_kernel<float, false, 4, 4>", "wide4")
    assert bench.kernel_name("f64", {"fused_steps": 1, "threads": 0}) == ("step_kernel<double, false, 1, 256>",
                                                                           "single")


def test_counter_means_separate_equal_thread_counts(tmp_path):
    """Two launch shapes with the same thread count but different workgroup
    sizes must not be averaged together."""
    d = tmp_path / "fetch"
    d.mkdir()
    name = "void ggfv::(anonymous namespace)::k<double, 2>(int)"
    rows = [{"Dispatch_Id": disp, "Kernel_Name": name, "Grid_Size": 8192, "Workgroup_Size": wg,
             "Counter_Name": "FETCH_SIZE", "Counter_Value": val}
            for disp, wg, val in ((1, 64, 10.0), (2, 64, 14.0), (3, 128, 100.0))]
    with open(d / "fetch_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    means = bench._counter_means(str(tmp_path), "fetch")
    assert means[("k<double, 2>", 8192, 64)] == pytest.approx(12.0)
    assert means[("k<double, 2>", 8192, 128)] == pytest.approx(100.0)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_copy_calibration_uses_the_largest_copies(tmp_path):
    """Copies of other sizes (checkpoints) run the same copy kernel in the same
    launch shape as the 1 GiB calibration copies; the calibration must come
    from the largest copy dispatches, not from the mean over all of them."""
    for kind, gib, small in (("fetch", 524288.0, 6144.0), ("write", 1048576.0, 12288.0)):
        d = tmp_path / kind
        d.mkdir()
        rows = []
        vals = [small] * 30 + [gib * 1.001, gib * 0.999, gib]
        for disp, val in enumerate(vals):
            rows.append({"Dispatch_Id": disp, "Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 4096,
                         "Workgroup_Size": 256, "Counter_Name": kind.upper() + "_SIZE", "Counter_Value": val})
        with open(d / f"{kind}_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=list(rows[0]))
            w.writeheader()
            w.writerows(rows)
    fetch, write = bench._counter_means(str(tmp_path), "fetch"), bench._counter_means(str(tmp_path), "write")
    _, f_scale, w_scale = bench._copy_calibration(fetch, write)
    assert f_scale == pytest.approx(2.0, rel=1e-3) and w_scale == pytest.approx(1.0, rel=1e-3)
