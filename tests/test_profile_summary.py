"""Host logic of the profile summaries (no GPU): the calibrated traffic record, the kernel-time
table and the per-kernel rates of the surrogate, on small synthetic rocprofv3 CSV files."""
import csv
import json

import pytest

from paper_1803_11345_amd import profile_summary as ps


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _counter_rows(counter, step_kib, copy_kib):
    rows = [{"Kernel_Name": "void k_step<ModeF32, 1, false, false>(...)", "Counter_Name": counter,
             "Counter_Value": v, "Grid_Size": 4096} for v in step_kib]
    # the probe copy at the largest grid, and a small copy that must be ignored
    rows += [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter, "Counter_Value": v,
              "Grid_Size": 1 << 20} for v in copy_kib]
    rows.append({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter, "Counter_Value": 1.0,
                 "Grid_Size": 64})
    return rows


def test_traffic_is_calibrated_by_the_copy(tmp_path):
    copy_bytes = 1 << 30
    # FETCH reads the copy at half its size (scale 2), WRITE at its size (scale 1)
    _write(tmp_path / "f.csv", _counter_rows("FETCH_SIZE", [1000.0, 1200.0], [copy_bytes / 2048.0] * 3))
    _write(tmp_path / "w.csv", _counter_rows("WRITE_SIZE", [900.0, 900.0], [copy_bytes / 1024.0] * 3))
    nodes, bpl = 100, 144
    rec = ps.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_step", copy_bytes, nodes, bpl, "cmd")
    assert rec["fetch"]["scale"] == pytest.approx(2.0) and rec["write"]["scale"] == pytest.approx(1.0)
    assert rec["fetch"]["copy_dispatches"] == 3 and rec["fetch"]["step_dispatches"] == 2
    fetch, write = 1100.0 * 1024 * 2, 900.0 * 1024
    assert rec["traffic_bytes_per_launch"] == pytest.approx(fetch + write)
    assert rec["traffic_over_algorithmic"] == pytest.approx((fetch + write) / (nodes * bpl))
    assert rec["read_over_algorithmic"] == pytest.approx(fetch / (nodes * bpl / 2))
    assert rec["source_sha256"] == ps.source_digest()
    json.dumps(rec)  # serialisable as written to profiles/


def test_traffic_without_the_kernel_fails(tmp_path):
    _write(tmp_path / "f.csv", _counter_rows("FETCH_SIZE", [1.0], [2.0]))
    with pytest.raises(SystemExit):
        ps.traffic(str(tmp_path / "f.csv"), str(tmp_path / "f.csv"), "k_missing", 1 << 20, 1, 1, "cmd")


def test_stats_and_rates_tables(tmp_path):
    stats = [{"Name": "_ZN12_GLOBAL__N_16k_convILi64ELi64ELi0ELb1EEEvPKDF16bS2_NS_7OutArgsEiii", "Calls": 4,
              "AverageNs": 40000.0, "MinNs": 39000.0, "MaxNs": 41000.0, "Percentage": 50.0},
             {"Name": "void (anonymous namespace)::k_last_dw<64>(bool _Accum const*, int)", "Calls": 1,
              "AverageNs": 20000.0, "MinNs": 20000.0, "MaxNs": 20000.0, "Percentage": 10.0}]
    _write(tmp_path / "s.csv", stats)
    md = ps.stats_md(str(tmp_path / "s.csv"), "the command")
    assert "| `k_conv<64, 64, 0>` | 4 | 40.00 | 39.00 | 41.00 | 50.00 % |" in md and "the command" in md
    counters = [{"Kernel_Name": stats[0]["Name"], "Counter_Name": "SQ_VALU_MFMA_BUSY_CYCLES", "Counter_Value": 256.0,
                 "Grid_Size": 1},
                {"Kernel_Name": stats[0]["Name"], "Counter_Name": "GRBM_GUI_ACTIVE", "Counter_Value": 8.0, "Grid_Size": 1}]
    _write(tmp_path / "c.csv", counters)
    md = ps.mfma_md(str(tmp_path / "s.csv"), str(tmp_path / "c.csv"), "cmds")
    flop, _, peak = ps.SURROGATE_WORK["k_conv<64, 64, 0>"]
    tf = flop / 40.0 / 1e6
    # busy 256 over (8 / 8 XCDs x 1024 SIMDs) = 0.25
    assert f"| `k_conv<64, 64, 0>` | 4 | 40.00 | {flop / 1e9:.2f} | {tf:.0f} | BF16 MFMA | {tf / peak:.3f} | 0.25 |" in md
    gbs = ps.SURROGATE_BYTES["k_last_dw<64>"] / 20.0 / 1e3
    assert f"| `k_last_dw<64>` | {ps.SURROGATE_BYTES['k_last_dw<64>'] / 1e6:.1f} | {gbs:.0f} | {gbs / 8000:.3f} |" in md
