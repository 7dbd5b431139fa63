"""The reducers of rocprofv3 output in paper_1907_11678_amd.profiling, on
small hand-made CSV files whose answers are known."""
from __future__ import annotations

import csv

import pytest

from paper_1907_11678_amd import profiling

SCAN = "void semb::scan_kernel<0, 15, 0>(semb::ScanArgs)"
COPY = "void __amd_rocclr_copyBuffer(...)"


def _counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, g, c, v in rows:
            w.writerow(dict(Dispatch_Id=d, Kernel_Name=k, Grid_Size=g, Counter_Name=c, Counter_Value=v))
    return str(path)


def test_traffic_record_uses_full_launches_and_the_copy_factor(tmp_path):
    # copy of 4 MiB: FETCH reads 2048 units (2048 B each), WRITE 4096 (1024 B each);
    # a small upload with the same copy kernel must not enter the factor
    fetch = _counters(tmp_path / "f.csv", [
        (1, COPY, 1024, "FETCH_SIZE", 2048.0), (2, COPY, 64, "FETCH_SIZE", 3.0),
        (3, SCAN, 1000, "FETCH_SIZE", 50.0),                                # tuner sample launch
        (4, SCAN, 8000, "FETCH_SIZE", 300.0), (4, SCAN, 8000, "FETCH_SIZE", 100.0),  # two dimensions
        (5, SCAN, 8000, "FETCH_SIZE", 400.0)])
    write = _counters(tmp_path / "w.csv", [
        (1, COPY, 1024, "WRITE_SIZE", 4096.0), (3, SCAN, 1000, "WRITE_SIZE", 5.0),
        (4, SCAN, 8000, "WRITE_SIZE", 10.0), (5, SCAN, 8000, "WRITE_SIZE", 30.0)])
    rec = profiling.traffic_record(fetch, write, "scan_kernel<0, 15, 0>", 4 << 20)
    assert rec["fetch_factor"] == pytest.approx(2048.0) and rec["write_factor"] == pytest.approx(1024.0)
    assert rec["fetch_kib_per_launch"] == pytest.approx(400.0) and rec["write_kib_per_launch"] == pytest.approx(20.0)
    assert rec["launches"] == 2
    assert rec["traffic_bytes_per_launch"] == pytest.approx(400.0 * 2048 + 20.0 * 1024)


def test_record_round_trip_and_digest_check(tmp_path, monkeypatch):
    rec = {"kernel": SCAN, "source_digest": profiling.source_digest(), "traffic_bytes_per_launch": 123.0}
    p = str(tmp_path / "rec.txt")
    profiling.write_record(rec, p, header="# a header line\n# kernel: not a field")
    assert profiling.current_traffic(p) == 123.0
    monkeypatch.setattr(profiling, "source_digest", lambda: "0000000000000000")
    assert profiling.current_traffic(p) is None
    assert profiling.current_traffic(str(tmp_path / "missing.txt")) is None


def test_rewriting_a_record_keeps_its_comment_header(tmp_path):
    p = str(tmp_path / "rec.txt")
    profiling.write_record({"traffic_bytes_per_launch": 1.0}, p, header="# line one\n#\n# line three")
    assert profiling.comment_header(p) == "# line one\n#\n# line three"
    assert profiling.comment_header(str(tmp_path / "none.txt")) == ""


def test_counter_summary_averages_full_launches_over_passes(tmp_path):
    evals = 64 * 1000  # 1000 64-lane evaluations per launch
    p1 = _counters(tmp_path / "p1.csv", [
        (1, SCAN, 100, "SQ_INSTS_VALU", 999.0),                  # small-grid launch: ignored
        (2, SCAN, 800, "SQ_INSTS_VALU", 50000.0), (3, SCAN, 800, "SQ_INSTS_VALU", 54000.0),
        (2, SCAN, 800, "SQ_LDS_IDX_ACTIVE", 4.0e5), (3, SCAN, 800, "SQ_LDS_IDX_ACTIVE", 6.0e5),
        (2, SCAN, 800, "GRBM_GUI_ACTIVE", 8 * 2000.0), (3, SCAN, 800, "GRBM_GUI_ACTIVE", 8 * 2000.0)])
    p2 = _counters(tmp_path / "p2.csv", [
        (7, SCAN, 800, "SQ_INSTS_VALU", 52000.0),                 # the same counter in a second pass
        (7, SCAN, 800, "SQ_INSTS_LDS_LOAD_BANDWIDTH", 4000.0),
        (7, SCAN, 800, "SQ_WAIT_ANY", 30.0), (7, SCAN, 800, "SQ_WAVE_CYCLES", 120.0),
        (7, SCAN, 800, "GRBM_GUI_ACTIVE", 8 * 1000.0)])
    out = profiling.counter_summary([p1, p2], "scan_kernel<0, 15, 0>", evals)
    per = out["counters_per_launch"]
    assert per["SQ_INSTS_VALU"] == pytest.approx(52000.0)      # (50000 + 54000 + 52000) / 3
    assert out["valu_insts_per_wave_eval"] == pytest.approx(52.0)
    assert out["gpu_cycles_per_launch"] == pytest.approx(1500.0)  # passes 2000 and 1000
    assert out["lds_busy_fraction"] == pytest.approx(5.0e5 / (1500.0 * 256))
    assert out["lds_load_bytes_per_lane_eval"] == pytest.approx(4000.0 * 64 / evals)
    assert out["wave_wait_fraction"] == pytest.approx(0.25)
    assert "GRBM_GUI_ACTIVE" not in per


def test_counter_summary_ignores_files_of_a_smaller_workload(tmp_path):
    # the same kernel on a smaller workload (a smaller grid) in another file
    # must not enter the per-launch average of the full workload's launches
    evals = 64 * 1000
    full = _counters(tmp_path / "full.csv", [
        (1, SCAN, 800, "SQ_INSTS_VALU", 52000.0), (1, SCAN, 800, "GRBM_GUI_ACTIVE", 8 * 2000.0)])
    small = _counters(tmp_path / "small.csv", [
        (4, SCAN, 80, "SQ_INSTS_VALU", 5200.0), (4, SCAN, 80, "GRBM_GUI_ACTIVE", 8 * 200.0)])
    out = profiling.counter_summary([small, full], "scan_kernel<0, 15, 0>", evals)
    assert out["counters_per_launch"]["SQ_INSTS_VALU"] == pytest.approx(52000.0)
    assert out["gpu_cycles_per_launch"] == pytest.approx(2000.0)
    with pytest.raises(SystemExit):
        profiling.counter_summary([small], "batch_kernel<11, 9, 0>", evals)


def test_kernel_trace_table_splits_by_grid(tmp_path):
    p = tmp_path / "t.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for g, ns in ((800, 3_000_000), (800, 5_000_000), (100, 1_000_000)):
            w.writerow(dict(Kernel_Name=SCAN, Grid_Size=g, Start_Timestamp=10, End_Timestamp=10 + ns))
    t = profiling.kernel_trace_table(str(p)).splitlines()
    assert t[2] == f"| `{SCAN}` | 800 | 2 | 4.000 | 3.000 | 5.000 |"
    assert t[3] == f"| `{SCAN}` | 100 | 1 | 1.000 | 1.000 | 1.000 |"
