"""The traffic summary of the committed profiles (prof_summary.traffic) on
synthetic rocprofv3 counter files: calibration by the device copy, kernels of
one span summed, and the name@grid filter that keeps one launch's dispatches
when the same kernel also runs with other grid sizes."""
import argparse
import csv
import json
import os

import pytest

from paper_2609_22608_amd import prof_summary as PS

COPY = "__amd_rocclr_copyBuffer"


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"])
        for name, grid, value in rows:
            w.writerow([name, counter, value, grid])


def _args(tmp_path, kernels, js):
    return argparse.Namespace(fetch=str(tmp_path / "f"), write=str(tmp_path / "w"), kernel=kernels,
                              key="edge_search", form="screen/3", grid=None, command="cmd",
                              json=js)


@pytest.fixture
def runs(tmp_path):
    # the 256 MiB copy: FETCH_SIZE reads half the bytes moved, WRITE_SIZE all
    cal_f, cal_w = 131072.0, 262144.0
    _write(tmp_path / "f", "FETCH_SIZE", [
        (COPY, 131072, cal_f), (COPY, 256, 1.0),
        ("void fn::tri_hist_kernel(int const*, long)", 8192, 100.0),
        ("void fn::tri_hist_kernel(int const*, long)", 8192, 120.0),
        ("void fn::tri_hist_kernel(int const*, long)", 256, 10.0),
        ("void fn::edge_search_open_kernel<5720, 1, true>(fn::EdgeArgs)", 2097152, 1000.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [
        (COPY, 131072, cal_w),
        ("void fn::tri_hist_kernel(int const*, long)", 8192, 8.0),
        ("void fn::tri_hist_kernel(int const*, long)", 256, 2.0),
        ("void fn::edge_search_open_kernel<5720, 1, true>(fn::EdgeArgs)", 2097152, 500.0)])
    return tmp_path


def test_span_sum_with_grid_filter(runs):
    js = str(runs / "t.json")
    PS.traffic(_args(runs, ["tri_hist_kernel@8192", "edge_search_open_kernel<5720, 1, true>"], js))
    rec = json.load(open(js))["edge_search"]
    # FETCH: (mean(100, 120) + 1000) KiB / 0.5; WRITE: (8 + 500) KiB / 1.0
    assert rec["fetch_scale"] == pytest.approx(0.5)
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["bytes_per_launch"] == pytest.approx(((110 + 1000) / 0.5 + 508) * 1024)
    assert rec["dispatches"] == [[2, 1], [1, 1]]
    assert rec["kernel"] == "tri_hist_kernel@8192 + edge_search_open_kernel<5720, 1, true>"


def test_without_filter_every_grid_counts(runs):
    js = str(runs / "t.json")
    PS.traffic(_args(runs, ["tri_hist_kernel"], js))
    rec = json.load(open(js))["edge_search"]
    assert rec["bytes_per_launch"] == pytest.approx(((100 + 120 + 10) / 3 / 0.5 + 5) * 1024)


def test_missing_kernel_or_grid_is_an_error(runs):
    with pytest.raises(SystemExit):
        PS.traffic(_args(runs, ["tri_hist_kernel@4096"], None))
    with pytest.raises(SystemExit):
        PS.traffic(_args(runs, ["no_such_kernel"], None))
