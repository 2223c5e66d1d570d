"""Host-side checks of the rocprofv3 summary tool (synthetic CSV, no GPU)."""
import csv
import json
import os

from paper_2412_06359_amd import profsum

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
        "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
        "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
        "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, COLS)
        w.writeheader()
        for i, (name, grid, val) in enumerate(rows):
            w.writerow({**{c: 0 for c in COLS}, "Dispatch_Id": i, "Grid_Size": grid,
                        "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val,
                        "Start_Timestamp": 1000 * i, "End_Timestamp": 1000 * i + 500})


def test_traffic_scaling(tmp_path):
    mib = 4
    _write(tmp_path / "cf", "FETCH_SIZE", [("copy_kernel(float4)", 10, mib * 512.0)])
    _write(tmp_path / "cw", "WRITE_SIZE", [("copy_kernel(float4)", 10, mib * 1024.0)])
    # two launch shapes of the kernel: the largest grid is the one summarised
    _write(tmp_path / "kf", "FETCH_SIZE", [("cm::bwd_sweep_kernel<2>", 100, 7.0),
                                           ("cm::bwd_sweep_kernel<2>", 900, 100.0),
                                           ("cm::bwd_sweep_kernel<2>", 900, 102.0)])
    _write(tmp_path / "kw", "WRITE_SIZE", [("cm::bwd_sweep_kernel<2>", 900, 8.0),
                                           ("cm::bwd_sweep_kernel<2>", 900, 8.0)])
    out = tmp_path / "t.json"
    profsum.main(["traffic", "--kernel", "bwd_sweep_kernel:adjoint", "--workload", "w",
                  "--fetch", str(tmp_path / "kf"), "--write", str(tmp_path / "kw"),
                  "--copy-fetch", str(tmp_path / "cf"), "--copy-write", str(tmp_path / "cw"),
                  "--copy-mib", str(mib), "--out", str(out)])
    rec = json.load(open(out))
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    ph = rec["phases"]["adjoint"]
    assert ph["grid"] == 900
    assert abs(ph["bytes_per_launch"] - (101.0 * 1024 * 2 + 8.0 * 1024)) < 1e-6
    assert (tmp_path / "t.md").exists()


def test_counter_table(tmp_path):
    # two counters of the same kernel in two runs; the largest grid is summarised
    _write(tmp_path / "a", "SQ_WAVE_CYCLES", [("cm::fwd_tile_own_kernel<256>", 50, 1.0),
                                              ("cm::fwd_tile_own_kernel<256>", 500, 1000.0),
                                              ("cm::fwd_tile_own_kernel<256>", 500, 3000.0)])
    _write(tmp_path / "b", "SQ_WAIT_ANY", [("cm::fwd_tile_own_kernel<256>", 500, 500.0),
                                           ("cm::fwd_tile_own_kernel<256>", 500, 1500.0)])
    out = tmp_path / "c.md"
    profsum.main(["counters", str(tmp_path / "a"), str(tmp_path / "b"), "--kernel",
                  "fwd_tile_own_kernel:splat", "--title", "T", "--cmd", "c1", "--out", str(out)])
    text = out.read_text()
    row = [l for l in text.splitlines() if l.startswith("| splat")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    # phase, kernel, grid, dispatches, SQ_WAIT_ANY, SQ_WAVE_CYCLES, wait/wave
    assert cells[2] == "500" and cells[3] == "2"
    assert float(cells[4]) == 1000.0 and float(cells[5]) == 2000.0
    assert abs(float(cells[6]) - 0.5) < 1e-12
