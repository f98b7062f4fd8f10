"""Host logic of the measurement tooling in bench.py (no GPU): the rocprofv3 summaries behind
profiles/ and the staleness rule for the recorded HBM traffic.  Synthetic CSVs with the
columns rocprofv3 writes stand in for real runs."""
import csv
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        for r in rows:
            w.writerow(r)


COUNTER_HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
                  "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
                  "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp",
                  "End_Timestamp"]
SPMM = ("void labpsd::(anonymous namespace)::k_spmm_hs<4>(long const*, int const*, double const*, double const*, "
        "long, long, double const*, long, int, int, int, double*, double*, long, labpsd::NlEpi<double, double>)")


def _counters(path, counter, values, name=SPMM):
    rows = [[i, i, "Agent 1", 1, 7, 7, 1024, 3, name, 512, 0, 0, 40, 0, 80, counter, float(v), 10 * i, 10 * i + 5]
            for i, v in enumerate(values)]
    _write_csv(path, COUNTER_HEADER, rows)


def test_short_kernel_name():
    assert bench.short_kernel_name(SPMM) == "k_spmm_hs<4>"
    assert bench.short_kernel_name('"void labpsd::(anonymous namespace)::k_gram<64, 32>(long, int)"') == \
        "k_gram<64,32>"
    assert bench.short_kernel_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"
    assert bench.kernel_source("k_sn_sweep<double,128,256>") == "paper_1308_2445_amd/csrc/precond.hip"
    assert bench.kernel_source("k_rrl_tridiag<true>") is None


def test_block_update_tile_width_follows_the_library():
    # the widths the library picks per launch (the block-update GPU test lists them)
    assert [bench.block_update_ct(b) for b in (40, 150, 130, 282, 128)] == [6, 6, 9, 9, 8]


def test_traffic_summary_and_staleness(tmp_path, monkeypatch):
    d = tmp_path / "pmc"
    # two dispatches of 100 and 300 KiB fetched, 50 KiB written each; calibration copies
    # of 512 MiB read 0.5 and write 1.0 of their bytes
    _counters(str(d / "fetch" / "vm" / "1_counter_collection.csv"), "FETCH_SIZE", [100.0, 300.0])
    _counters(str(d / "write" / "vm" / "1_counter_collection.csv"), "WRITE_SIZE", [50.0, 50.0])
    _counters(str(d / "cf" / "vm" / "1_counter_collection.csv"), "FETCH_SIZE", [262144.0], "__amd_rocclr_copyBuffer")
    _counters(str(d / "cw" / "vm" / "1_counter_collection.csv"), "WRITE_SIZE", [524288.0], "__amd_rocclr_copyBuffer")
    out = tmp_path / "profiles" / "hbm_traffic_test.txt"
    out.parent.mkdir()
    bench.summarize_traffic([str(d / "fetch"), str(d / "write"), str(d / "cf"), str(d / "cw")], str(out), "cmd")
    lines = [l for l in open(out) if l.startswith("kernel=")]
    assert len(lines) == 1
    f = dict(kv.split("=", 1) for kv in lines[0].split())
    assert f["kernel"] == "k_spmm_hs<4>" and f["dispatches"] == "2"
    assert float(f["fetch_factor"]) == pytest.approx(0.5) and float(f["write_factor"]) == pytest.approx(1.0)
    # (200 KiB / 0.5 + 50 KiB / 1.0) per launch
    assert int(f["bytes_per_launch"]) == (400 + 50) * 1024
    src = os.path.join(ROOT, "paper_1308_2445_amd", "csrc", "spmm.hip")
    assert f["sha256"] == bench.source_digest(src)
    # the bench reads it back while the digest matches, and not once it does not
    monkeypatch.setattr(bench, "PROFILE_DIR", str(out.parent))
    assert bench.measured_traffic("k_spmm_hs<4>", "test") == (400 + 50) * 1024
    assert bench.measured_traffic("k_gram<64,32>", "test") is None
    text = open(out).read().replace(f["sha256"], "0" * 64)
    open(out, "w").write(text)
    assert bench.measured_traffic("k_spmm_hs<4>", "test") is None


def test_source_digest_covers_the_shared_header(tmp_path):
    csrc = tmp_path / "csrc"
    csrc.mkdir()
    (csrc / "k.hip").write_text("kernel\n")
    (csrc / "common.h").write_text("helpers v1\n")
    a = bench.source_digest(str(csrc / "k.hip"))
    (csrc / "common.h").write_text("helpers v2\n")
    assert bench.source_digest(str(csrc / "k.hip")) != a


def test_stats_summary(tmp_path):
    header = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"]
    rows = [["void labpsd::(anonymous namespace)::k_residual(long, int)", 4, 4000.0, 1000.0, 20.0, 900, 1100, 10.0],
            ["void labpsd::(anonymous namespace)::k_gram<64, 32>(long)", 2, 16000.0, 8000.0, 80.0, 7000, 9000, 5.0]]
    _write_csv(str(tmp_path / "prof" / "vm" / "1_kernel_stats.csv"), header, rows)
    out = tmp_path / "stats.txt"
    bench.summarize_stats(str(tmp_path / "prof"), str(out), "cmd")
    body = [l.split() for l in open(out) if l.startswith("k_")]
    assert [b[0] for b in body] == ["k_gram<64,32>", "k_residual"]   # by total time
    assert body[0][1] == "2" and float(body[0][3]) == pytest.approx(8.0)
    assert "total kernel time 0.0 ms" in open(out).read()


def test_apply_levels_summary(tmp_path):
    header = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
              "Correlation_Id", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
              "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z",
              "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]

    def k(name, t0, t1, tasks):
        return ["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, 1, 1, "void labpsd::(anonymous namespace)::%s(int)" % name,
                1, t0, t1, 0, 0, 64, 0, 64, 256, 1, 1, 256 * tasks, 1, 1]
    # one sweep, then one level-by-level apply: two forward levels, the diagonal, two backward
    rows = [k("k_sn_sweep<double, 128, 256>", 0, 9000, 40),
            k("k_sn_product<double, 2>", 10000, 11000, 8), k("k_sn_product<double, 2>", 11000, 11500, 2),
            k("k_sn_product<double, 0>", 11500, 12500, 10),
            k("k_sn_product<double, 3>", 12500, 13000, 2), k("k_sn_product<double, 3>", 13000, 14000, 8)]
    _write_csv(str(tmp_path / "prof" / "vm" / "1_kernel_trace.csv"), header, rows)
    out = tmp_path / "levels.txt"
    bench.summarize_apply_levels(str(tmp_path / "prof"), str(out), "cmd")
    text = open(out).read()
    assert "double single-launch sweep: 9.0 us (40 work-groups)" in text
    assert "double level by level: 5 launches, 4.0 us of kernels, 4.0 us first start to last end" in text
    table = [l.split() for l in text.splitlines() if l.split() and l.split()[0] in ("forward", "diagonal", "backward")]
    assert [(r[0], r[1], r[2]) for r in table] == [("forward", "0", "8"), ("forward", "1", "2"), ("diagonal", "0", "10"),
                                                   ("backward", "0", "2"), ("backward", "1", "8")]
