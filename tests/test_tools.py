"""Host logic of the measurement tools on synthetic rocprofv3 CSV files: the
HBM-traffic reduction of the FETCH_SIZE / WRITE_SIZE passes (scaled by what
the counters read for a device copy of known size, largest launches of each
class only) and the step summary (per-step HBM, algorithmic and FP64
figures, wave states)."""
import csv
import json
import os

import pytest

from paper_1810_04597_amd import profsum, traffic

UPDATE = "void grmhd::k_update_zm<grmhd::FlatMet<double>, 2, 6, double, 3>(grmhd::Geom, double const*)"
SWEEP = "void grmhd::k_sweep_lds<1, 4, grmhd::FlatMet<double>, double, 0>(grmhd::Geom)"
COPY = "__amd_rocclr_copyBuffer"
GiB = 1 << 30


def _counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, grid, ctr, val) in enumerate(rows):
            w.writerow([i, grid, name, ctr, val])


def test_traffic_scaling_and_largest_launches(tmp_path):
    """FETCH reads half of the copied bytes and WRITE all of them: factors 2
    and 1; a class's bytes are the mean over its largest-grid launches."""
    kib = GiB / 1024
    _counters(tmp_path / "f", [(COPY, 1 << 20, "FETCH_SIZE", kib / 2), (COPY, 256, "FETCH_SIZE", 5.0),
                               (UPDATE, 65536, "FETCH_SIZE", 1000.0), (UPDATE, 65536, "FETCH_SIZE", 3000.0),
                               (UPDATE, 1024, "FETCH_SIZE", 7.0)])
    _counters(tmp_path / "w", [(COPY, 1 << 20, "WRITE_SIZE", kib), (UPDATE, 65536, "WRITE_SIZE", 400.0)])
    res = traffic.compute(str(tmp_path / "f"), str(tmp_path / "w"), GiB)
    assert res["fetch_scale"] == pytest.approx(2.0) and res["write_scale"] == pytest.approx(1.0)
    u = res["kernels"]["update"]
    assert u["fetch_bytes"] == pytest.approx(2000.0 * 2 * 1024)
    assert u["write_bytes"] == pytest.approx(400.0 * 1024)
    assert u["bytes"] == pytest.approx(u["fetch_bytes"] + u["write_bytes"])
    out = tmp_path / "t.json"
    traffic.main(str(tmp_path / "f"), str(tmp_path / "w"), GiB, out=str(out))
    assert json.load(open(out))["kernels"]["update"]["bytes"] == pytest.approx(u["bytes"])


def test_step_summary_figures(tmp_path):
    """Three launches per stage kernel per step: 3 x (6 + 3) GB over 20 ms is
    1.35 TB/s; the copy of 1 GiB in 0.4 ms reads and writes 2 GiB; FP64
    FLOP = 64 (ADD + MUL + 2 FMA) per wavefront instruction."""
    kt = tmp_path / "kt"
    os.makedirs(kt)
    with open(kt / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "AverageNs"])
        w.writerow([UPDATE, 33, 1.5e6])
        w.writerow([SWEEP, 33, 0.8e6])
    with open(kt / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"])
        w.writerow([COPY, 1 << 20, 1000, 1000 + 400000])
        w.writerow([COPY, 1 << 20, 5000000, 5000000 + 500000])
    tj = tmp_path / "traffic.json"
    json.dump({"source_hash": "x", "fetch_scale": 2.0, "write_scale": 1.0,
               "kernels": {"update": {"bytes": 6e9}, "sweep_x2": {"bytes": 3e9}}}, open(tj, "w"))
    _counters(tmp_path / "v", [(n, 65536, c, val) for n in (UPDATE, SWEEP) for c, val in (
        ("SQ_INSTS_VALU_ADD_F64", 1e6), ("SQ_INSTS_VALU_MUL_F64", 2e6), ("SQ_INSTS_VALU_FMA_F64", 3e6),
        ("SQ_INSTS_VALU_TRANS_F64", 0.0), ("SQ_INSTS_VALU", 2e7))])
    _counters(tmp_path / "s", [(n, 65536, c, val) for n in (UPDATE, SWEEP) for c, val in (
        ("SQ_WAVE_CYCLES", 1000.0), ("SQ_WAIT_ANY", 300.0), ("SQ_WAIT_INST_ANY", 400.0),
        ("SQ_ACTIVE_INST_ANY", 300.0), ("SQ_ACTIVE_INST_VALU", 200.0), ("SQ_ACTIVE_INST_LDS", 10.0),
        ("SQ_LDS_BANK_CONFLICT", 0.0))])
    bench = tmp_path / "bench.log"
    bench.write_text("warmup\n" + json.dumps({"ms_per_step": 20.0, "value": 8.4e8, "launch": "graph"}) + "\n")
    out = tmp_path / "p.md"
    profsum.main(["--ktrace", str(kt), "--valu", str(tmp_path / "v"), "--stall", str(tmp_path / "s"),
                  "--bench", str(bench), "--traffic", str(tj), "--out", str(out)])
    text = out.read_text()
    assert "27.0 GB per step" in text and "= 1.35 TB/s" in text
    copy_rate = 2 * GiB / 0.4e-3
    assert "%.2f TB/s a plain 1 GiB device copy" % (copy_rate / 1e12) in text
    assert "= 0.753 TB/s" in text                     # 896 B x 8.4e8/s
    f64 = 2 * 3 * 64.0 * (1e6 + 2e6 + 2 * 3e6)       # two classes, three launches each
    assert "%.1f TFLOP/s" % (f64 / 0.02 / 1e12) in text
    assert "| update | 0.30 | 0.40 | 0.30 | 0.20 | 0.010 | 0 |" in text
    assert "| update (stage 2, in place) | 33 | 1500.0 | 6.00 |" in text
