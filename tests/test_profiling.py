"""Host logic of the rocprofv3 summaries (paper_1411_0127_amd/profiling.py) on
synthetic CSV files: only the dispatches between the two marker fills count as
the timed region, and the traffic scale comes from the calibration copies made
after it, not from other copies of the program (the autotuner copies spins)."""
import csv
import json

import pytest

from paper_1411_0127_amd import profiling

SWEEP = "void sg::(anonymous namespace)::k_fused2<0, 5>(sg::(anonymous namespace)::FusedParams)"
MARK = "void sg::(anonymous namespace)::k_probe_fill<false>(HIP_vector_type<unsigned int, 4u>*, unsigned long, unsigned int)"
COPY = "__amd_rocclr_copyBuffer"


def write_trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, t0, t1 in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": t0, "End_Timestamp": t1})


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": k + 1, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_trace_counts_only_the_timed_region(tmp_path):
    rows = [(SWEEP, 0, 9000)]                       # an autotuner candidate, slow
    rows += [(MARK, 10000, 10001)]
    rows += [(SWEEP, 10100 + 2000 * k, 10100 + 2000 * k + 1000) for k in range(4)]  # four 1000 ns launches
    rows += [(MARK, 20000, 20001), (SWEEP, 30000, 38000)]
    p = tmp_path / "trace.csv"
    write_trace(p, rows)
    out = profiling.trace(str(p), str(tmp_path / "t.md"), "cmd")
    text = open(out).read()
    timed = text.split("All dispatches")[0]
    assert "4 dispatches" in timed
    assert "| `sg::k_fused2<0, 5>` | 4 | 1.00 |" in timed
    assert "| `sg::k_fused2<0, 5>` | 6 |" in text.split("All dispatches")[1]


def test_traffic_scale_from_the_calibration_copies(tmp_path):
    copy_bytes = 1 << 30
    # FETCH_SIZE counts the copy's reads as half their size, WRITE_SIZE exactly
    fetch = [(COPY, 4 * 1048576.0), (SWEEP, 99.0), (MARK, 0.0), (SWEEP, 1000.0), (SWEEP, 1002.0), (MARK, 0.0),
             (COPY, copy_bytes / 2048.0), (COPY, copy_bytes / 2048.0)]
    write = [(COPY, 8 * 1048576.0), (SWEEP, 7.0), (MARK, 0.0), (SWEEP, 300.0), (SWEEP, 300.0), (MARK, 0.0),
             (COPY, copy_bytes / 1024.0), (COPY, copy_bytes / 1024.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fp, "FETCH_SIZE", fetch)
    write_counters(wp, "WRITE_SIZE", write)
    out = profiling.traffic(str(fp), str(wp), "cx", copy_bytes, "cmd <COUNTER>", out_dir=str(tmp_path))
    rec = json.load(open(out))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_kib_per_launch_raw"] == pytest.approx(1001.0)   # timed launches only
    assert rec["hbm_read_bytes_per_launch"] == pytest.approx(1001.0 * 1024 * 2)
    assert rec["hbm_write_bytes_per_launch"] == pytest.approx(300.0 * 1024)
    assert rec["command_fetch"] == "cmd FETCH_SIZE"


def test_traffic_needs_the_markers(tmp_path):
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fp, "FETCH_SIZE", [(SWEEP, 1.0), (COPY, 1.0)])
    write_counters(wp, "WRITE_SIZE", [(SWEEP, 1.0), (COPY, 1.0)])
    with pytest.raises(SystemExit):
        profiling.traffic(str(fp), str(wp), "cx", 1 << 30, "cmd", out_dir=str(tmp_path))


def test_valu_record_counts_the_timed_launches(tmp_path):
    rows = []
    for k, (name, insts, cyc) in enumerate([(SWEEP, 5.0, 9.0), (MARK, 0.0, 1.0), (SWEEP, 100.0, 50.0),
                                            (SWEEP, 102.0, 52.0), (SWEEP, 101.0, 51.0), (MARK, 0.0, 1.0),
                                            (SWEEP, 7.0, 3.0)]):
        rows.append({"Dispatch_Id": k + 1, "Kernel_Name": name, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": insts})
        rows.append({"Dispatch_Id": k + 1, "Kernel_Name": name, "Counter_Name": "GRBM_GUI_ACTIVE", "Counter_Value": cyc})
    p = tmp_path / "v.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        w.writerows(rows)
    out = profiling.valu(str(p), "cx", "cmd", "fused2,16,16,0,1,5", out_dir=str(tmp_path))
    assert out.endswith("valu_sweep_fused_cx_fused2_16_16_0_1_5.json")
    rec = json.load(open(out))
    assert rec["valu_wave_insts_per_launch"] == 101.0 and rec["gui_active_cycles_per_launch"] == 51.0
    assert rec["launches"] == 3 and rec["tile"] == ["fused2", 16, 16, 0, 1, 5]
