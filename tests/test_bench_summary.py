"""Host logic of bench.py's rocprofv3 summary (the source of the files in
profiles/): grouping by kernel and launch shape, the dominant mixed-mode
evaluation's dispatches in launch order, the stats table, and the
copy-calibrated byte counts of the counter passes."""
import csv
import os

import bench


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_kernel_trace_summary(tmp_path, capsys):
    d = tmp_path / "kt"
    d.mkdir()
    hdr = ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Workgroup_Size_X", "Start_Timestamp",
           "End_Timestamp"]
    mixed = "void nb::(anonymous namespace)::force_kernel<0, 1, 4, false, false>(x)"
    rows = [[mixed, 65536, 16, 256, 0, 2_000_000],          # 2 ms
            ["nb::sched_min(x)", 4096, 1, 256, 3_000_000, 3_005_000],
            [mixed, 65536, 16, 256, 4_000_000, 10_000_000],  # 6 ms
            [mixed, 65536, 16, 256, 11_000_000, 15_000_000],  # 4 ms
            # a later, shorter mixed evaluation of another shape (a microbenchmark
            # size): the dominant shape is the one with the largest total time
            [mixed, 32768, 1, 256, 16_000_000, 19_000_000]]  # 3 ms
    _write(d / "kt_kernel_trace.csv", hdr, rows)
    _write(d / "kt_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"],
           [[mixed, 3, 12_000_000, 4_000_000], ["nb::sched_min(x)", 1, 5000, 5000]])
    bench.summarize_profile(str(d))
    out = capsys.readouterr().out
    line = [l for l in out.splitlines() if "force_kernel<0, 1, 4" in l and "x 16" in l][0]
    calls, total, avg, med = line.split()[:4]
    assert (int(calls), float(total), float(avg), float(med)) == (3, 12.0, 4.0, 4.0)
    assert "grid 65536 x 16: 3 dispatches in launch order (ms): 2.0000 6.0000 4.0000" in out
    assert "--stats" in out and "12.000" in out


def test_counter_calibration(tmp_path, capsys):
    d = tmp_path / "f"
    d.mkdir()
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value",
           "Start_Timestamp", "End_Timestamp"]
    mixed = "void nb::(anonymous namespace)::force_kernel<0, 1, 4, false, false>(x)"
    rows = [[4, "__amd_rocclr_copyBuffer", 131072, "FETCH_SIZE", 524288, 0, 400_000],
            [9, mixed, 1048576, "FETCH_SIZE", 1000, 500_000, 7_000_000]]
    _write(d / "f_counter_collection.csv", hdr, rows)
    bench.summarize_profile(str(d))
    out = capsys.readouterr().out
    # 1 GiB copy counts 524288 KiB -> factor 2; 1000 KiB -> 2.048 MB
    assert "factor 2.0000" in out and "-> 2.05 MB per launch" in out


def test_read_traffic(tmp_path, monkeypatch):
    """roofline.traffic comes from the two copy-calibrated counter lines of
    the committed summary; the kernel's name and grid come with it."""
    f = tmp_path / "c.txt"
    name = "void nb::force_kernel<0, 1, 4, false, false, 2>"
    f.write_text(
        f"# FETCH_SIZE: 1 GiB copy (dispatch 4) counts 524300 KiB -> factor 2.0000; dominant kernel "
        f"dispatch 52 ({name}, grid 524288, 923.932 ms) 2.59993e+06 KiB -> 5324.53 MB per launch\n"
        f"# WRITE_SIZE: 1 GiB copy (dispatch 4) counts 1.04858e+06 KiB -> factor 1.0000; dominant "
        f"kernel dispatch 52 ({name}, grid 524288, 922.122 ms) 81920 KiB -> 83.89 MB per launch\n")
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(f))
    tot, kern = bench.read_traffic()
    assert abs(tot - 5408.42e6) < 1.0 and kern == (name, 524288)
    f.write_text("nothing here\n")
    assert bench.read_traffic() is None
