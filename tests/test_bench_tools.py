"""CPU tests of bench.py's rocprofv3 summarizers on small synthetic csv files:
the HBM traffic per launch of the opposite-spin kernel (counter mean x the
copy-calibration factor, FETCH_SIZE + WRITE_SIZE), its gating by the kernel
source hash, and the per-kernel counter means."""
import csv
import os

import bench

KNAME = "void tbsci::(anonymous namespace)::k_ab_slab<double, 20>(long, int)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, name, rows):
    os.makedirs(d, exist_ok=True)
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
           "End_Timestamp"]
    _write(os.path.join(d, "x_counter_collection.csv"), hdr,
           [[i, k, name, v, 1000 * i, 1000 * i + dur] for i, (k, v, dur) in enumerate(rows)])


def test_summarize_traffic_and_hash_gate(tmp_path, monkeypatch):
    trace = tmp_path / "trace"
    trace.mkdir()
    _write(trace / "x_kernel_stats.csv",
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"],
           [[KNAME, 2, 6000000, 3000000, 90.0, 2900000, 3100000]])
    # copy of 256 MiB: FETCH_SIZE reads half of it (factor 2), WRITE_SIZE all (factor 1)
    _counters(str(tmp_path / "fetch"), "FETCH_SIZE",
              [(COPY, 131072.0, 5), (KNAME, 1000.0, 7), (KNAME, 3000.0, 7)])
    _counters(str(tmp_path / "write"), "WRITE_SIZE",
              [(COPY, 262144.0, 5), (KNAME, 500.0, 7), (KNAME, 500.0, 7)])
    out = tmp_path / "summary.txt"
    bench.summarize(str(trace), str(tmp_path / "fetch"), str(tmp_path / "write"), str(out),
                    ["cmd"])
    text = out.read_text()
    expect = 2000 * 1024 * 2 + 500 * 1024 * 1  # KiB per dispatch x factor, fetch + write
    assert f"traffic opposite_spin fp64 {expect} k_ab_slab<double,20>" in text
    assert "fetch_factor 2.0000 write_factor 1.0000" in text
    monkeypatch.setattr(bench, "PROFILE", str(out))
    assert bench.measured_traffic("opposite_spin", "fp64") == (expect, "k_ab_slab<double,20>")
    assert bench.measured_traffic("opposite_spin", "fp32") == (None, None)
    monkeypatch.setattr(bench, "source_hash", lambda: "changed")
    assert bench.measured_traffic("opposite_spin", "fp64") == (None, None)


def test_summarize_title_and_ambiguous_kernels(tmp_path):
    """The summary header is the profiled workload's title, and a run in
    which two kernels serve the same term and precision is refused (its
    traffic could not be attributed)."""
    import pytest
    trace = tmp_path / "trace"
    trace.mkdir()
    K2 = "void tbsci::(anonymous namespace)::k_ab_slabg<double, 24, 2>(long, int)"
    _write(trace / "x_kernel_stats.csv",
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"],
           [[KNAME, 1, 3000000, 3000000, 50.0, 3000000, 3000000]])
    _counters(str(tmp_path / "fetch"), "FETCH_SIZE",
              [(COPY, 131072.0, 5), (KNAME, 1000.0, 7)])
    _counters(str(tmp_path / "write"), "WRITE_SIZE",
              [(COPY, 262144.0, 5), (KNAME, 500.0, 7)])
    out = tmp_path / "s.txt"
    bench.summarize(str(trace), str(tmp_path / "fetch"), str(tmp_path / "write"), str(out),
                    ["cmd"], "my workload title")
    assert out.read_text().startswith("# rocprofv3 summary: my workload title")
    _counters(str(tmp_path / "fetch2"), "FETCH_SIZE",
              [(COPY, 131072.0, 5), (KNAME, 1000.0, 7), (K2, 10.0, 7)])
    _counters(str(tmp_path / "write2"), "WRITE_SIZE",
              [(COPY, 262144.0, 5), (KNAME, 500.0, 7), (K2, 10.0, 7)])
    with pytest.raises(SystemExit):
        bench.summarize(str(trace), str(tmp_path / "fetch2"), str(tmp_path / "write2"),
                        str(tmp_path / "s2.txt"), ["cmd"])


def test_summarize_counters_means(tmp_path):
    d = str(tmp_path / "pmc")
    _counters(d, "SQ_BUSY_CYCLES", [(KNAME, 10.0, 2000), (KNAME, 30.0, 4000)])
    out = tmp_path / "c.txt"
    bench.summarize_counters(d, str(out), ["cmd"], "t")
    text = out.read_text()
    assert "k_ab_slab<double, 20>  dispatches 2  mean_us 3.0" in text
    assert "SQ_BUSY_CYCLES                   2.000000e+01" in text
