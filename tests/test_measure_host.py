"""Host logic of the measurement helpers (no GPU): matching a rocprofv3
kernel trace to a launch plan, turning two counter passes into HBM bytes per
launch, and the read shapes of the bench's quick read floor."""

import csv
import json
import math

import pytest

from paper_2501_10653_amd import measure


def _write_trace(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for name, s, e in rows:
            w.writerow([name, s, e])


def test_trace_summary_assigns_dispatches_to_segments_in_order(tmp_path):
    # Two segments of tiles_kernel launches with fills and copies in between,
    # written out of start order: the summary walks them in start order and
    # skips the kernels a segment does not name.
    rows = [("tiles_kernel<4,4,8,3>", 100 + 10 * i, 100 + 10 * i + d)
            for i, d in enumerate([7, 9, 8])]                        # segment A: 7, 9, 8
    rows += [("fill_kernel", 95, 99), ("copyBuffer", 135, 138)]
    rows += [("tiles_kernel<4,4,8,3>", 200 + 10 * i, 200 + 10 * i + d)
             for i, d in enumerate([5, 6, 4, 30])]                    # segment B: 5, 6, 4, 30
    rows.reverse()
    trace = tmp_path / "t.csv"
    _write_trace(trace, rows)
    plan = measure.Plan()
    plan.add("A", "tiles_kernel", 3, bytes=800)
    plan.add("B", "tiles_kernel", 4)
    plan_path = tmp_path / "p.json"
    plan.dump(str(plan_path))
    a, b = measure.trace_summary(str(trace), str(plan_path))
    assert a["label"] == "A" and a["dispatches"] == 3 and a["expected"] == 3
    assert a["median_ns"] == 8 and a["min_ns"] == 7 and a["mean_ns"] == 8 and a["bytes"] == 800
    assert b["dispatches"] == 4 and b["median_ns"] == 5.5 and b["min_ns"] == 4
    assert b["p90_ns"] == pytest.approx(6 + 0.7 * (30 - 6))     # numpy's linear p90


def test_trace_summary_reports_missing_dispatches(tmp_path):
    trace = tmp_path / "t.csv"
    _write_trace(trace, [("tiles_kernel", 0, 5)])
    plan = measure.Plan()
    plan.add("A", "tiles_kernel", 2)
    plan.add("B", "tiles_kernel", 1)
    p = tmp_path / "p.json"
    plan.dump(str(p))
    a, b = measure.trace_summary(str(trace), str(p))
    assert a["dispatches"] == 1 and a["expected"] == 2
    assert b["dispatches"] == 0 and "median_ns" not in b


def _write_counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Counter_Value"])
        for name, v in rows:
            w.writerow([name, v])


def test_traffic_scales_each_counter_by_the_copy_calibration(tmp_path):
    cal_kib = measure.CALIBRATION_BYTES / 1024
    # FETCH counts half the bytes of the 256 MiB copies (scale 2), WRITE all
    # of them (scale 1); small copies before them do not calibrate.
    fetch = [("copyBuffer", 3.0), ("tiles_kernel", 1000.0), ("tiles_kernel", 1002.0)]
    fetch += [("copyBuffer", cal_kib / 2)] * 3
    write = [("tiles_kernel", 8.0), ("tiles_kernel", 8.0)] + [("copyBuffer", cal_kib)] * 3
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counters(f, fetch)
    _write_counters(w, write)
    t = measure.traffic(str(f), str(w), "tiles_kernel", 2_000_000)
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["fetch_kib_per_dispatch"] == 1001.0 and t["fetch_dispatches"] == 2
    assert t["hbm_bytes_per_launch"] == (1001 * 2 + 8) * 1024
    assert t["ratio"] == pytest.approx((1001 * 2 + 8) * 1024 / 2_000_000, abs=1e-5)


def test_traffic_needs_the_kernel_and_the_calibration(tmp_path):
    f = tmp_path / "f.csv"
    _write_counters(f, [("tiles_kernel", 1.0)])
    with pytest.raises(ValueError):
        measure.traffic(str(f), str(f), "tiles_kernel", 1)


def test_quick_read_shapes_issue_all_their_loads_on_32_mib():
    n4 = (32 << 20) // 16
    for mode, blocks, threads, loads in measure.QUICK_READS:
        assert mode in measure.READ_MODES
        assert threads % 64 == 0 and 64 <= threads <= 1024
        assert loads in (4, 8, 16, 32)
        # every lane's loads in flight fall inside its workgroup's chunk
        assert math.ceil(n4 / blocks) >= loads * threads
        if mode == 2:
            assert loads * threads * 16 <= 64 * 1024       # dynamic LDS of the LDS form


def test_plan_dump_round_trips(tmp_path):
    plan = measure.Plan()
    plan.add("x (warm)", "probe_read_regs<", 5, bytes=16)
    p = tmp_path / "p.json"
    plan.dump(str(p))
    assert json.load(open(p)) == {"segments": [{"label": "x (warm)", "kernel": "probe_read_regs<",
                                                "count": 5, "bytes": 16}]}


def test_timeline_stats_splits_a_launch_into_ramp_data_tail_and_gap():
    import numpy as np
    launches, nwg = 3, 4
    rec = np.zeros((launches, nwg, 8), dtype=np.int64)
    for L in range(launches):
        for w in range(nwg):
            entry = 1000 * L + w
            last = entry + 300 + 10 * w
            rec[L, w] = [entry, entry + 100, last, last + 20, w % 8, 0, w, 1 << 32]
    t = measure.timeline_stats(rec, khz=100_000, event_us=9.5, bytes_launch=3_330_000)
    tick = 0.01                                   # µs per tick at 100 MHz
    assert t["workgroups"] == nwg and t["launches"] == launches
    assert t["dispatch_ramp_us"]["median"] == pytest.approx(3 * tick)
    assert t["first_data_us"]["median"] == pytest.approx(100 * tick)
    assert t["last_data_us"]["median"] == pytest.approx(333 * tick)
    assert t["tail_us"]["median"] == pytest.approx(20 * tick)
    assert t["span_us"]["median"] == pytest.approx(353 * tick)
    assert t["gap_to_next_launch_us"]["median"] == pytest.approx((1000 - 353) * tick)
    assert t["finishing_wg_exit_after_data_us"]["median"] == pytest.approx(20 * tick)
    assert t["other_wg_exit_after_data_us"] is None
    assert t["workgroups_per_xcd"][:4] == [1, 1, 1, 1]
    assert t["data_phase_GBs"] == pytest.approx(3_330_000 / 3.33 / 1e3)
    assert t["event_us_per_launch"] == 9.5
