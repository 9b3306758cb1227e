"""The rocprofv3 counter digest (paper_2203_05871_amd.counters): per-dispatch
sums, the dispatch window, and the copy calibration, on a small synthetic
counter file in rocprofv3's CSV layout."""
import csv
import json

from paper_2203_05871_amd import counters

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, name, counter, value in rows:
            w.writerow({k: 0 for k in FIELDS} | {"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
                                                  "Counter_Value": value})


def test_window_sums_and_copy_scale(tmp_path):
    # dispatch 1: the calibration copy (reads half of its size); dispatches 2..7 the kernel, one of
    # them reported in two rows that must be summed; a foreign kernel in between
    fetch = tmp_path / "fetch.csv"
    write_csv(fetch, [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0),
                      (2, "void k<false>(X)", "FETCH_SIZE", 10.0),
                      (3, "void k<false>(X)", "FETCH_SIZE", 20.0),
                      (4, "other", "FETCH_SIZE", 1e6),
                      (5, "void k<false>(X)", "FETCH_SIZE", 30.0),
                      (5, "void k<false>(X)", "FETCH_SIZE", 6.0),
                      (6, "void k<false>(X)", "FETCH_SIZE", 40.0),
                      (7, "void k<false>(X)", "FETCH_SIZE", 1000.0)])
    write = tmp_path / "write.csv"
    write_csv(write, [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0)] +
              [(d, "void k<false>(X)", "WRITE_SIZE", 8.0) for d in (2, 3, 5, 6, 7)])
    out = tmp_path / "rec.json"
    # the window: the 3 kernel dispatches before the last one
    counters.main(["--kernel", "k<", "--pass", f"FETCH_SIZE={fetch}", "--pass", f"WRITE_SIZE={write}",
                   "--copy-kib", "1024", "--window", "3", "--skip-tail", "1", "--out", str(out)])
    rec = json.loads(out.read_text())
    assert rec["launches_averaged"] == 3 and rec["launches_in_run"] == 5
    assert rec["FETCH_SIZE_per_launch_raw"] == (20.0 + 36.0 + 40.0) / 3
    assert rec["FETCH_SIZE_scale"] == 2.0 and rec["WRITE_SIZE_scale"] == 1.0
    assert rec["hbm_bytes_per_launch"] == ((20.0 + 36.0 + 40.0) / 3 * 2.0 + 8.0) * 1024.0


def test_source_hash_changes_with_the_source(tmp_path):
    f = tmp_path / "fetch.csv"
    write_csv(f, [(1, "k", "FETCH_SIZE", 1.0)])
    src = tmp_path / "a.hip"
    src.write_text("one")
    out = tmp_path / "r.json"
    args = ["--kernel", "k", "--pass", f"FETCH_SIZE={f}", "--source", "a.hip", "--root", str(tmp_path),
            "--out", str(out)]
    counters.main(args)
    h1 = json.loads(out.read_text())["source_sha256"]
    src.write_text("two")
    counters.main(args)
    assert json.loads(out.read_text())["source_sha256"] != h1
