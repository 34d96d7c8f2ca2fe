"""Host logic of the rocprofv3 summaries (paper_2510_01764_amd.profile_summary)
on small synthetic CSV files of rocprofv3's column layout: the kernel-statistics
table with the per-dispatch median, the HBM-traffic scaling by the calibration
copy, and the vector-ALU count per launch."""
import csv
import json
import os

import pytest

from paper_2510_01764_amd import profile_summary as PS

FUSED = "void octax::(anonymous namespace)::step_fused_kernel<256, true, false, false>(octax::State, octax::Roms)"
COPY = "octax_calib_copy_kernel(uint4 const*, uint4*, unsigned long)"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _trace(d, durations):
    rows, t = [], 1000
    for name, ns in durations:
        rows.append([name, t, t + ns])
        t += ns + 10
    _write(os.path.join(d, "x_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)


def test_stats_table_has_the_dispatch_median(tmp_path):
    d = str(tmp_path / "prof")
    # five launches of the fused kernel: one slow outlier pulls the mean, not the median
    durs = [7_500_000, 7_400_000, 10_000_000, 7_600_000, 7_510_000]
    _trace(d, [(FUSED, x) for x in durs] + [(COPY, 500_000), (COPY, 520_000)])
    _write(os.path.join(d, "x_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"],
           [[FUSED, 5, sum(durs), sum(durs) / 5, 97.0, min(durs), max(durs)],
            [COPY, 2, 1_020_000, 510_000, 3.0, 500_000, 520_000]])
    out = str(tmp_path / "stats.txt")
    PS.stats(d, out, "python bench.py")
    lines = open(out).read().splitlines()
    assert lines[1] == "# command: python bench.py"
    assert lines[3].split() == ["kernel", "calls", "avg_us", "median_us", "min_us", "max_us", "total_ms", "pct"]
    row = lines[4].split()
    # the short name keeps the template arguments and drops namespace and parameters
    assert " ".join(row[:4]) == "step_fused_kernel<256, true, false, false>"
    assert row[4:] == ["5", "8002.0", "7510.0", "7400.0", "10000.0", "40.01", "97.00"]
    copy = lines[5].split()
    assert copy[0] == "octax_calib_copy_kernel" and copy[3] == "510.0"   # even count: mean of the middle two


def _counters(d, counter, values):
    _write(os.path.join(d, "v_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
           [[k, counter, v] for k, v in values])


def test_traffic_scales_by_the_calibration_copy(tmp_path):
    fd, wd = str(tmp_path / "f"), str(tmp_path / "w")
    C = 1 << 30
    # the copy's counters read 2x (fetch) and 1x (write) its true size in KiB
    _counters(fd, "FETCH_SIZE", [(COPY, 2 * C / 1024), (FUSED, 100.0), (FUSED, 300.0)])
    _counters(wd, "WRITE_SIZE", [(COPY, C / 1024), (FUSED, 1000.0), (FUSED, 1000.0)])
    out = str(tmp_path / "t.json")
    PS.traffic(fd, wd, out, C, "step_fused_kernel<256, true, false, false>", "f", "w")
    d = json.load(open(out))
    assert d["scale_fetch"] == pytest.approx(0.5) and d["scale_write"] == pytest.approx(1.0)
    assert d["hbm_fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 0.5)
    assert d["hbm_write_bytes_per_launch"] == pytest.approx(1000.0 * 1024)
    assert d["dispatches"] == [2, 2]


def test_valu_is_the_mean_per_dispatch_times_64_lanes(tmp_path):
    d = str(tmp_path / "v")
    _counters(d, "SQ_INSTS_VALU", [(FUSED, 100.0), (FUSED, 300.0), (COPY, 5.0)])
    out = str(tmp_path / "v.json")
    PS.valu(d, out, "step_fused_kernel<256, true, false, false>", "cmd")
    r = json.load(open(out))
    assert r["valu_insts_per_dispatch"] == 200.0 and r["dispatches"] == 2
    assert r["valu_lane_ops_per_launch"] == 200.0 * 64


def test_ambiguous_kernel_name_is_an_error(tmp_path):
    d = str(tmp_path / "v")
    _counters(d, "SQ_INSTS_VALU", [(FUSED, 1.0), (FUSED.replace("true, false, false", "false, false, false"), 2.0)])
    with pytest.raises(SystemExit):
        PS.valu(d, str(tmp_path / "o.json"), "step_fused_kernel<256", "cmd")


def test_bench_reads_counter_summaries_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16
    t, v = tmp_path / "t.json", tmp_path / "v.json"
    t.write_text(json.dumps({"kernel_source_hash": h, "hbm_bytes_per_launch": 123.0}))
    v.write_text(json.dumps({"kernel_source_hash": h, "valu_lane_ops_per_launch": 456.0,
                             "active_lane_fraction": 0.75}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(t))
    monkeypatch.setattr(bench, "VALU_FILE", str(v))
    assert bench.measured_traffic() == 123.0 and bench.measured_valu() == 456.0
    assert bench.measured_active_lanes() == 0.75
    # a summary of another source version, or an unreadable one, gives null
    t.write_text(json.dumps({"kernel_source_hash": "0" * 16, "hbm_bytes_per_launch": 123.0}))
    v.write_text("not json")
    assert bench.measured_traffic() is None and bench.measured_valu() is None
    assert bench.measured_active_lanes() is None


def test_lanes_adds_the_active_lane_fraction(tmp_path, monkeypatch):
    import bench
    d = str(tmp_path / "l")
    os.makedirs(d)
    _write(os.path.join(d, "l_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
           [[FUSED, "SQ_THREAD_CYCLES_VALU", 4800.0], [FUSED, "SQ_ACTIVE_INST_VALU", 100.0],
            [FUSED, "SQ_THREAD_CYCLES_VALU", 4800.0], [FUSED, "SQ_ACTIVE_INST_VALU", 100.0]])
    out = tmp_path / "v.json"
    out.write_text(json.dumps({"kernel_source_hash": bench.kernel_source_hash(), "valu_lane_ops_per_launch": 1.0}))
    PS.lanes(d, str(out), "step_fused_kernel<256, true, false, false>", "cmd")
    r = json.load(open(out))
    assert r["valu_active_lanes"] == 48.0 and r["active_lane_fraction"] == 0.75
    assert r["valu_lane_ops_per_launch"] == 1.0          # the VALU count is kept
    out.write_text(json.dumps({"kernel_source_hash": "0" * 16}))
    with pytest.raises(SystemExit):
        PS.lanes(d, str(out), "step_fused_kernel<256, true, false, false>", "cmd")
