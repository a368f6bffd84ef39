"""bench.py's counter summary on the host: rocprofv3 --pmc CSV files of a plain
copy and of a solve are folded into HBM bytes per launch (scaled by what the
counter reads for the copy) and into bytes per round of the last solve."""

import csv
import json
import os

import pytest

bench = pytest.importorskip("bench")

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_run(d, counter, rows):
    os.makedirs(d)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for i, (name, kib) in enumerate(rows, 1):
            w.writerow([i, i, "Agent 1", 1, 1, 1, 64, 1, f"void mstx::{name}(mstx::ScanArgs)", 64, 0, 0, 8, 0, 8,
                        counter, kib, 0, 1])


def test_summary_scales_and_splits_rounds(tmp_path):
    mib = 256
    copy = [("__amd_rocclr_copyBuffer", mib * 1024 / 2), ("__amd_rocclr_copyBuffer", mib * 1024 / 2)]
    write_run(str(tmp_path / "cf"), "FETCH_SIZE", copy)  # the copy's reads, counted at half
    write_run(str(tmp_path / "cw"), "WRITE_SIZE", [(n, 2 * v) for n, v in copy])
    # two solves; the second one's rounds: (scan, bucket_min, hook, compress, finalize, relabel), (scan, tail)
    one = [("k_init", 1), ("k_scan<2, 0>", 100), ("k_bucket_min", 50), ("k_hook", 10), ("k_compress", 4),
           ("k_finalize", 1), ("k_relabel", 3), ("k_scan<1, 3>", 40), ("k_round_tail", 2)]
    fetch = one + [(n, 2 * v) for n, v in one]
    write_run(str(tmp_path / "sf"), "FETCH_SIZE", fetch)
    write_run(str(tmp_path / "sw"), "WRITE_SIZE", [(n, 1.0) for n, _ in fetch])
    out = tmp_path / "summary.json"
    doc = bench.summarize_pmc(str(tmp_path / "cf"), str(tmp_path / "cw"), str(tmp_path / "sf"), str(tmp_path / "sw"),
                              mib, "random_n1M_d16", out_path=str(out))
    assert json.load(open(out)) == doc
    cal = doc["copy_calibration"]
    assert cal["fetch_factor"] == pytest.approx(2.0) and cal["write_factor"] == pytest.approx(1.0)
    k = doc["kernels"]["k_scan<2, 0>"]
    # FETCH KiB 100 and 200 over the two solves, x2 calibration; WRITE 1 KiB each
    assert k["launches"] == 2
    assert k["fetch_bytes_mean"] == pytest.approx(1.5 * 100 * 1024 * 2)
    assert k["write_bytes_mean"] == pytest.approx(1024)
    rounds = doc["per_round_last_solve"]
    assert [sorted(r) for r in rounds] == [sorted(["k_scan<2, 0>", "k_bucket_min", "k_hook", "k_compress",
                                                   "k_finalize", "k_relabel"]),
                                           sorted(["k_scan<1, 3>", "k_round_tail"])]
    assert rounds[1]["k_scan<1, 3>"]["fetch_bytes"] == pytest.approx(80 * 1024 * 2)
    assert rounds[0]["k_hook"]["traffic_bytes"] == pytest.approx(20 * 1024 * 2 + 1024)
