"""Host-side checks of the rocprofv3 summaries (no GPU): the traffic scaling
by the calibration copy and the matrix-core busy fraction, on small synthetic
counter tables written in rocprofv3's CSV columns."""
import csv

import pytest

from paper_1910_06409_amd import profiling

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
        "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
        "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
        "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _table(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=COLS)
        w.writeheader()
        for disp, name, counter, value, t0, t1 in rows:
            r = {c: 0 for c in COLS}
            r.update(Dispatch_Id=disp, Kernel_Name=name, Counter_Name=counter,
                     Counter_Value=value, Start_Timestamp=t0, End_Timestamp=t1, Grid_Size=512)
            w.writerow(r)


def _agent(path, simds=1024, xcc=8):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Node_Id", "Agent_Type", "Simd_Count", "Num_Xcc"])
        w.writerow([0, "CPU", 0, 1])
        w.writerow([1, "GPU", simds, xcc])


def test_mfma_summary_busy_fraction_and_clock(tmp_path):
    # two dispatches of the rank-k kernel, 2.0e6 ns each; 8 XCDs active for
    # 4.0e6 cycles each (2.0 GHz); MFMA busy 1024 SIMDs x 3.0e6 cycles (0.75)
    sym = "void gke::k_rankk_f64(gke::cx<double> const*, int)"
    rows = []
    for disp in (5, 9):
        t0 = 1_000_000 * disp
        rows += [(disp, sym, "GRBM_GUI_ACTIVE", 8 * 4.0e6, t0, t0 + 2_000_000),
                 (disp, sym, "SQ_VALU_MFMA_BUSY_CYCLES", 1024 * 3.0e6, t0, t0 + 2_000_000),
                 (disp, sym, "SQ_WAVES", 1000, t0, t0 + 2_000_000)]
    # another kernel's rows are ignored
    rows.append((7, "void gke::k_rankk_rem<gke::cx<double>, false>(int)", "GRBM_GUI_ACTIVE",
                 1.0, 0, 10))
    _table(tmp_path / "c.csv", rows)
    _agent(tmp_path / "a.csv")
    text = profiling.mfma_summary(str(tmp_path / "c.csv"), str(tmp_path / "a.csv"), "fp64",
                                  "w", "cmd")
    d = {}
    for line in text.splitlines():
        if not line.startswith("#") and ":" in line:
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    assert d["kernel"] == "k_rankk_f64"
    assert int(d["dispatches"]) == 2
    assert float(d["mfma_busy_fraction"]) == pytest.approx(0.75)
    assert float(d["clock_ghz"]) == pytest.approx(2.0)
    assert float(d["mfma_busy_cycles_per_wave"]) == pytest.approx(1024 * 3.0e6 / 1000, rel=1e-6)
    assert d["source_hash"] == profiling.source_hash("rankk")


def test_traffic_summary_scales_by_the_copy(tmp_path):
    # the copy of 1 MiB reads 1024 KiB of FETCH_SIZE (factor 1) and 512 KiB of
    # WRITE_SIZE (factor 2); the kernel reads 300 and 100 KiB per dispatch
    copy = "__amd_rocclr_copyBuffer"
    sym = "void gke::k_fin_kz(double const*)"
    _table(tmp_path / "f.csv", [(1, copy, "FETCH_SIZE", 1024.0, 0, 1),
                                (2, copy, "FETCH_SIZE", 4.0, 0, 1),
                                (3, sym, "FETCH_SIZE", 300.0, 0, 1)])
    _table(tmp_path / "w.csv", [(1, copy, "WRITE_SIZE", 512.0, 0, 1),
                                (3, sym, "WRITE_SIZE", 100.0, 0, 1)])
    text = profiling.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                                     "fin_kz", "fp64", 1 << 20, "f", "w", "x")
    p = tmp_path / "t.txt"
    p.write_text(text)
    d = profiling.read_summary(str(p))
    assert float(d["fetch_factor"]) == pytest.approx(1.0)
    assert float(d["write_factor"]) == pytest.approx(2.0)
    assert profiling.traffic_if_current(str(p), "fin_kz", "fp64") == pytest.approx(
        300 * 1024 + 2 * 100 * 1024)
    assert profiling.traffic_if_current(str(p), "fin_kx", "fp64") is None
