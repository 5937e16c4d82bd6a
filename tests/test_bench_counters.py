"""The benchmark's counter reducers on synthetic rocprofv3 counter files
(no GPU): bytes per launch group from FETCH_SIZE / WRITE_SIZE scaled by the
calibration copy, the choice of one kernel instance by precision and
template argument, and the markdown counter table."""
import csv
import json
import os

import pytest

import bench

CAL = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(at::TensorIteratorBase&)>(int)"
XCB64 = "void xab::(anonymous namespace)::k_spmv_xcb<double, double, double, 32>(xab::XcbArgs, double const*)"
XCB32 = "void xab::(anonymous namespace)::k_spmv_xcb<float, float, double, 16>(xab::XcbArgs, float const*)"
FIX = "void xab::(anonymous namespace)::k_xcb_fixup<double>(xab::XcbArgs, long)"
COMB64 = "void xab::(anonymous namespace)::k_xcb_combine<double, double>(xab::XcbArgs, unsigned char const*)"
COMB32 = "void xab::(anonymous namespace)::k_xcb_combine<float, double>(xab::XcbArgs, unsigned char const*)"


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


@pytest.fixture
def runs(tmp_path):
    cal_kib = bench.CAL_BYTES / 1024
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    # the copy reads half its bytes in FETCH_SIZE units and writes all of them
    _write(f, [(CAL, "FETCH_SIZE", cal_kib / 2)] +
           [(XCB64, "FETCH_SIZE", v) for v in (1000.0, 1200.0)] + [(XCB32, "FETCH_SIZE", 600.0)] +
           [(FIX, "FETCH_SIZE", 2.0), (COMB64, "FETCH_SIZE", 100.0), (COMB32, "FETCH_SIZE", 90.0)])
    _write(w, [(CAL, "WRITE_SIZE", cal_kib)] +
           [(XCB64, "WRITE_SIZE", 50.0), (XCB32, "WRITE_SIZE", 40.0), (FIX, "WRITE_SIZE", 1.0),
            (COMB64, "WRITE_SIZE", 20.0), (COMB32, "WRITE_SIZE", 10.0)])
    return f, w, tmp_path


def test_pmc_summary_scales_by_the_calibration_copy(runs):
    f, w, tmp = runs
    out = str(tmp / "t.json")
    bench.pmc_summary(f, w, out, "XCB", 100, "cf", "cw")
    rep = json.load(open(out))
    assert rep["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert rep["calibration"]["write_factor"] == pytest.approx(1.0)
    k = rep["kernels"]
    # FP64 instances only; the mean over dispatches, times 1024 times the factor
    assert k["k_spmv_xcb"]["read_bytes"] == pytest.approx(1100.0 * 1024 * 2)
    assert k["k_spmv_xcb"]["dispatches"] == [2, 1]
    assert k["k_xcb_combine"]["write_bytes"] == pytest.approx(20.0 * 1024)
    tot = rep["traffic_bytes_per_spmv"]
    assert tot["read"] == pytest.approx((1100.0 + 2.0 + 100.0) * 2048)
    assert tot["write"] == pytest.approx((50.0 + 1.0 + 20.0) * 1024)
    assert tot["total"] == pytest.approx(tot["read"] + tot["write"])
    assert rep["source_sha256"] == bench.spmv_source_hash("XCB")


def test_pmc_summary_fp32_instances(runs):
    f, w, tmp = runs
    out = str(tmp / "t32.json")
    bench.pmc_summary(f, w, out, "XCB", 100, "cf", "cw", precision="f32")
    k = json.load(open(out))["kernels"]
    assert "float, float, double, 16" in k["k_spmv_xcb"]["name"]
    assert "float, double" in k["k_xcb_combine"]["name"]
    assert "fixup<double>" in k["k_xcb_fixup"]["name"]  # shared by both precisions


def test_pick_instance_rules():
    names = [XCB64, XCB32, "void xab::k_spmv_xcb<double, double, double, 4>(x)"]
    with pytest.raises(SystemExit):
        bench._pick_instance(names, "k_spmv_xcb", "f64", "")  # two FP64 instances
    assert bench._pick_instance(names, "k_spmv_xcb", "f64", ", 32>") == XCB64
    assert bench._pick_instance(names, "k_spmv_xcb", "f32", "") == XCB32
    with pytest.raises(SystemExit):
        bench._pick_instance(names, "k_spmv_sell", "f64", "")


def test_missing_reading_is_an_error(runs, tmp_path):
    f, _, tmp = runs
    w2 = str(tmp_path / "w2")
    _write(w2, [(CAL, "WRITE_SIZE", bench.CAL_BYTES / 1024)])
    with pytest.raises(SystemExit):
        bench.pmc_summary(f, w2, str(tmp / "x.json"), "XCB", 100, "cf", "cw")


def test_counter_summary_table(runs):
    f, w, tmp = runs
    out = str(tmp / "c.md")
    bench.counter_summary([f, w], out, "XCB", 100, 1000, ["cmd a", "cmd b"])
    text = open(out).read()
    assert "cmd a" in text and "## `k_spmv_xcb`" in text
    assert "| FETCH_SIZE | 1,100 |" in text and "| WRITE_SIZE | 50 |" in text
