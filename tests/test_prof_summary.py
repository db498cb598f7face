"""The rocprofv3 summariser beside bench.py (host only): kernel statistics,
per-dispatch averages with the short/long split, counter averages with the
calibration copy kept, and --delete removing only the per-dispatch files."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import prof_summary  # noqa: E402


def _write(path, header, rows):
    with open(path, "w") as f:
        f.write(",".join(header) + "\n")
        for r in rows:
            f.write(",".join(str(v) for v in r) + "\n")


def test_trace_split_and_stats(tmp_path, capsys):
    d = tmp_path / "run"
    (d / "host").mkdir(parents=True)
    _write(d / "host" / "x_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [["k_dslash<a>", 3, 1710000, 570000, 90.0], ["other", 1, 5, 5, 10.0]])
    _write(d / "host" / "x_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp",
                                               "Workgroup_Size_X", "Grid_Size_X"],
           [["k_dslash<a>", 0, 10000, 256, 256], ["k_dslash<a>", 0, 800000, 256, 256],
            ["k_dslash<a>", 0, 900000, 256, 256], ["other", 0, 5, 64, 64]])
    prof_summary.main([str(d), "--match", "k_dslash", "--split-us", "100", "--delete"])
    out = capsys.readouterr().out
    assert "3 | 1.710 | 570.00 | 90.00 | k_dslash<a>" in out
    assert "dispatches: 3; average 570.00 us; min 10.00 us; max 900.00 us" in out
    assert "shorter than 100 us: 1; average 10.00 us" in out
    assert "100 us or longer: 2; average 850.00 us; min 800.00 us; max 900.00 us" in out
    assert not (d / "host" / "x_kernel_trace.csv").exists()
    assert (d / "host" / "x_kernel_stats.csv").exists()


def test_counter_averages_keep_the_copy(tmp_path, capsys):
    d = tmp_path / "pmc"
    d.mkdir()
    rows = []
    for disp, (name, v) in enumerate((("k_dslash<b>", 10.0), ("k_dslash<b>", 30.0), ("__amd_rocclr_copyBuffer", 7.0),
                                      ("unrelated", 1.0))):
        for inst in range(2):   # two hardware instances per dispatch, summed
            rows.append([disp, name, "FETCH_SIZE", v / 2])
    _write(d / "p_counter_collection.csv", ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    prof_summary.main([str(d), "--match", "k_dslash"])
    out = capsys.readouterr().out
    assert "FETCH_SIZE | dispatches 2 | avg 20.0 | min 10.0 | max 30.0 | k_dslash<b>" in out
    assert "FETCH_SIZE | dispatches 1 | avg 7.0 | min 7.0 | max 7.0 | __amd_rocclr_copyBuffer" in out
    assert "unrelated" not in out
