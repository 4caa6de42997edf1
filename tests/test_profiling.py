"""The profile summaries bench.py reads its roofline figures from: the
summariser on small synthetic rocprofv3 CSV files (kernel trace and counter
collection, in rocprofv3's column layout), the copy calibration of the byte
counters, the launch window, and bench.py's use of the figures (the
algorithmic fraction from the profiled duration, traffic as read + write,
stale figures ignored)."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1304_7126_amd import profiling  # noqa: E402

TRACE_COLS = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
              "Correlation_Id", "Start_Timestamp", "End_Timestamp"]
PMC_COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
            "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def write_csv(path, cols, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow({c: r.get(c, 0) for c in cols})


def trace(tmp_path):
    # ten launches of k_chem_all of 1000 + 10 k us each, interleaved with a
    # transport kernel, out of time order in the file
    rows, t, d = [], 1000, 1
    for k in range(10):
        rows.append({"Dispatch_Id": d, "Kernel_Name": "void rtm1::k_transport_z<float, 1, 768, true>(...)",
                     "Start_Timestamp": t, "End_Timestamp": t + 500_000})
        t += 600_000
        d += 1
        rows.append({"Dispatch_Id": d, "Kernel_Name": "void rtm1::k_chem_all<float, 3, 0>(...)",
                     "Start_Timestamp": t, "End_Timestamp": t + 1_000_000 + 10_000 * k})
        t += 2_000_000
        d += 1
    rows.reverse()
    p = tmp_path / "trace.csv"
    write_csv(p, TRACE_COLS, rows)
    return p


def pmc(tmp_path, name, counter, per_dispatch, copy_value):
    # each dispatch's counter split over two rows (per-instance values that
    # the summariser adds up), plus three 1 GiB copies
    rows, d = [], 1
    for v in per_dispatch:
        for half in (0.25 * v, 0.75 * v):
            rows.append({"Dispatch_Id": d, "Kernel_Name": "void rtm1::k_chem_all<float, 3, 0>(...)",
                         "Counter_Name": counter, "Counter_Value": half})
        d += 1
    for _ in range(3):
        rows.append({"Dispatch_Id": d, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter,
                     "Counter_Value": copy_value})
        d += 1
    p = tmp_path / name
    write_csv(p, PMC_COLS, rows)
    return p


def test_stats_window_and_average(tmp_path):
    out = tmp_path / "stats.md"
    profiling.stats(str(trace(tmp_path)), str(out), ["cmd"], "k_chem_all", 3, 5, "t")
    f = profiling.read_figures(str(out))
    # launches 3..7 in time order last 1000 + 10 k us for k = 2..6
    assert f["window"] == [3, 7]
    assert f["avg_us"] == pytest.approx(1040.0)
    assert f["kernel_source_hash"] == profiling.kernel_source_hash()
    assert "rtm1::k_chem_all<float, 3, 0>" in f["kernel"]


def test_bytes_are_scaled_by_the_copy(tmp_path):
    gib = 1 << 30
    # the copy reads FETCH_SIZE of half its bytes and WRITE_SIZE of all
    fetch = pmc(tmp_path, "fetch.csv", "FETCH_SIZE", [100.0, 200.0, 300.0, 400.0], gib / 1024 / 2)
    write = pmc(tmp_path, "write.csv", "WRITE_SIZE", [50.0, 60.0, 70.0, 80.0], gib / 1024)
    out = tmp_path / "bytes.md"
    profiling.bytes_(str(fetch), str(write), str(out), ["cmd"], "k_chem_all", 2, 2, "t", copy_bytes=gib)
    f = profiling.read_figures(str(out))
    assert f["fetch_scale"] == pytest.approx(2.0) and f["write_scale"] == pytest.approx(1.0)
    assert f["read_bytes"] == pytest.approx(250.0 * 1024 * 2)
    assert f["write_bytes"] == pytest.approx(65.0 * 1024)
    assert f["window"] == [2, 3]


def test_counters_average_every_counter(tmp_path):
    p = pmc(tmp_path, "valu.csv", "SQ_INSTS_VALU", [10.0, 20.0, 30.0], 0.0)
    out = tmp_path / "valu.md"
    profiling.counters(str(p), str(out), ["cmd"], "k_chem_all", 1, 3, "t")
    f = profiling.read_figures(str(out))
    assert f["SQ_INSTS_VALU"] == pytest.approx(20.0)
    assert f["window"] == [1, 3]


def test_bench_roofline_uses_current_profiles_and_ignores_stale_ones(tmp_path):
    import bench
    prefix = str(tmp_path / "k_chem_all_x")
    # a summary set taken with the current sources
    for kind, fig in (("_kernel_stats.md", {"avg_us": 4000.0}),
                      ("_pmc_bytes.md", {"read_bytes": 3e9, "write_bytes": 2e9}),
                      ("_pmc_valu.md", {"SQ_INSTS_VALU": 1.2e9, "SQ_ACTIVE_INST_VALU": 1.0e9,
                                        "SQ_THREAD_CYCLES_VALU": 48e9, "SQ_WAIT_ANY": 1e9, "SQ_WAVE_CYCLES": 4e9})):
        profiling._write(prefix + kind, "t", ["cmd"], "body", {"window": [11, 110], **fig})
    nbytes = 168 * 256 ** 3
    r = bench.kernel_roofline("k_chem_all", nbytes, 4.1, prefix, (11, 110), True)
    assert r["profile"]["status"] == "ok"
    assert r["frac"] == pytest.approx(nbytes / 4.1e-3 / 1e9 / 8000.0)
    assert r["profile"]["frac_from_profile"] == pytest.approx(nbytes / 4.0e-3 / 1e9 / 8000.0)
    assert r["traffic"] == pytest.approx(5e9)
    assert r["alu"]["valu_issue_frac"] == pytest.approx(1.2e9 / 4.0e-3 / bench.VALU_ISSUE_PEAK)
    assert r["alu"]["lane_util"] == pytest.approx(0.75)
    # another launch window: not used
    r = bench.kernel_roofline("k_chem_all", nbytes, 4.1, prefix, (1, 100), True)
    assert r["traffic"] is None and "alu" not in r
    # summaries of other kernel sources: not used
    with open(prefix + "_pmc_bytes.md") as f:
        text = f.read()
    with open(prefix + "_pmc_bytes.md", "w") as f:
        f.write(text.replace(profiling.kernel_source_hash(), "0" * 16))
    r = bench.kernel_roofline("k_chem_all", nbytes, 4.1, prefix, (11, 110), True)
    assert r["traffic"] is None and r["traffic_status"].startswith("kernel sources changed")


def test_committed_profiles_parse():
    import bench
    windows = {"": [11, 110], "_launches6to25": [6, 25]}
    for prefix in (bench.PROFILE, bench.PROFILE_TRANSPORT):
        assert len(bench.PROFILE_SETS[prefix]) == len(windows)
        for cand in bench.PROFILE_SETS[prefix]:
            suffix = cand[len(prefix):]
            for kind in ("_kernel_stats.md", "_pmc_bytes.md", "_pmc_valu.md", "_pmc_mix.md"):
                f = profiling.read_figures(cand + kind)
                assert f is not None, cand + kind
                assert f["window"] == windows[suffix]
                assert len(f["kernel_source_hash"]) == 16
                json.dumps(f)


def test_bench_picks_the_profile_set_of_its_window(tmp_path, monkeypatch):
    import bench
    prefix = str(tmp_path / "k_chem_all_x")
    for p, win, us in ((prefix, [11, 110], 4000.0), (prefix + "_launches6to25", [6, 25], 3000.0)):
        profiling._write(p + "_kernel_stats.md", "t", ["cmd"], "body", {"window": win, "avg_us": us})
    monkeypatch.setitem(bench.PROFILE_SETS, prefix, [prefix, prefix + "_launches6to25"])
    nbytes = 168 * 256 ** 3
    assert bench.kernel_roofline("k", nbytes, 3.0, prefix, (6, 25), True)["profile"]["avg_us"] == 3000.0
    assert bench.kernel_roofline("k", nbytes, 4.0, prefix, (11, 110), True)["profile"]["avg_us"] == 4000.0
    assert bench.kernel_roofline("k", nbytes, 4.0, prefix, (1, 50), True)["traffic"] is None
