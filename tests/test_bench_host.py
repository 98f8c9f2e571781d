"""Host logic of bench.py (no GPU): the one-GPU refusal, the gate that reports HBM traffic only
while the kernel sources match the counter record, and the rocprofv3 summaries (kernel
statistics; FETCH_SIZE / WRITE_SIZE calibrated on a plain copy of known size)."""
import csv
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_csv(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _pmc_rows(counter, lean_parts, copies):
    """Counter rows as rocprofv3 writes them: one row per (dispatch, instance); the summary adds
    the instances of a dispatch."""
    lean = "void lf::k_maps_tile<false>(lf::MapsArgs)"
    rows, d = [], 0
    for parts in lean_parts:
        d += 1
        for v in parts:
            rows.append({"Dispatch_Id": d, "Kernel_Name": lean, "Counter_Name": counter, "Counter_Value": v})
    for v in copies:
        d += 1
        rows.append({"Dispatch_Id": d, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter,
                     "Counter_Value": v})
    # another kernel's dispatches are ignored
    rows.append({"Dispatch_Id": d + 1, "Kernel_Name": "lf::k_expand(...)", "Counter_Name": counter,
                 "Counter_Value": 1e9})
    return rows


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_pmc_summary_calibrates_on_the_copy(tmp_path, capsys):
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    kib = bench.COPY_PROBE_BYTES / 1024
    # FETCH_SIZE reads half of the copy's bytes (factor 2); the three largest copies are the probe
    _write_csv(str(tmp_path / "f" / "run" / "run_counter_collection.csv"), fields,
               _pmc_rows("FETCH_SIZE", [[60.0, 40.0], [120.0]], [kib / 2] * 3 + [5.0]))
    # WRITE_SIZE counts all of them (factor 1)
    _write_csv(str(tmp_path / "w" / "run" / "run_counter_collection.csv"), fields,
               _pmc_rows("WRITE_SIZE", [[50.0], [30.0, 40.0]], [kib] * 3 + [7.0]))
    bench.summarize_profiles("pmc", [str(tmp_path / "f"), str(tmp_path / "w")])
    out = capsys.readouterr().out.strip().splitlines()
    rec = json.loads(out[-1])
    assert rec["copy_factor_fetch"] == pytest.approx(2.0)
    assert rec["copy_factor_write"] == pytest.approx(1.0)
    assert rec["dispatches"] == 2
    assert rec["fetch_bytes_per_launch"] == pytest.approx(110.0 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(60.0 * 1024)
    assert rec["source_sha256"] == bench.kernel_source_hash()


def test_stats_summary_lists_every_kernel(tmp_path, capsys):
    fields = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"]
    rows = [{"Name": "void lf::k_maps_tile<false>(lf::MapsArgs)", "Calls": 4, "TotalDurationNs": 4.4e6,
             "AverageNs": 1.1e6, "Percentage": 80.0},
            {"Name": "lf::k_expand(...)", "Calls": 2, "TotalDurationNs": 1.1e6, "AverageNs": 5.5e5,
             "Percentage": 20.0}]
    _write_csv(str(tmp_path / "s" / "x" / "step_kernel_stats.csv"), fields, rows)
    bench.summarize_profiles("stats", [str(tmp_path / "s")])
    lines = capsys.readouterr().out.strip().splitlines()
    assert lines[0] == "# source_sha256: " + bench.kernel_source_hash()
    assert lines[1].split() == ["kernel", "calls", "avg_us", "total_ms", "pct"]
    first = lines[2].split()
    assert first[-4:] == ["4", "1100.00", "4.400", "80.00"]
    assert len(lines) == 4


def test_profile_timing_is_reported_only_for_the_recorded_sources(tmp_path, monkeypatch):
    f = tmp_path / "stats.txt"
    row = "void %s(lf::MapsArgs)" % bench.LEAN_KERNEL
    f.write_text("# header\n# source_sha256: %s\nkernel calls avg_us total_ms pct\n%-60s %7d %12.2f %12.3f %7.2f\n"
                 % (bench.kernel_source_hash(), row, 70, 726.39, 50.847, 25.84))
    monkeypatch.setattr(bench, "STATS_FILE", str(f))
    assert bench.recorded_profile_ms() == pytest.approx(0.72639)
    f.write_text(f.read_text().replace(bench.kernel_source_hash(), "0" * 64))
    assert bench.recorded_profile_ms() is None


def test_traffic_is_reported_only_for_the_recorded_sources(tmp_path, monkeypatch):
    good = {"kernel": "lf::k_maps_tile<false>", "source_sha256": bench.kernel_source_hash(),
            "fetch_bytes_per_launch": 3.0e8, "write_bytes_per_launch": 1.5e8}
    f = tmp_path / "traffic.txt"
    f.write_text("# header\n" + json.dumps(good) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic() == pytest.approx(4.5e8)
    stale = dict(good, source_sha256="0" * 64)
    f.write_text("# header\n" + json.dumps(stale) + "\n")
    assert bench.recorded_traffic() is None
    f.write_text("# no record\n")
    assert bench.recorded_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.recorded_traffic() is None


def test_committed_traffic_record_is_well_formed():
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    assert rec["kernel"] == "lf::k_maps_tile<false>"
    assert rec["fetch_bytes_per_launch"] > 0 and rec["write_bytes_per_launch"] > 0
    for k in ("copy_factor_fetch", "copy_factor_write"):
        assert 0.5 <= rec[k] <= 4.0
    assert len(rec["source_sha256"]) == 64


def test_flops_summary_joins_counters_and_times(tmp_path, capsys):
    sfields = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"]
    _write_csv(str(tmp_path / "s" / "x" / "x_kernel_stats.csv"), sfields,
               [{"Name": "kA", "Calls": 2, "TotalDurationNs": 2e6, "AverageNs": 1e6, "Percentage": 90},
                {"Name": "kB", "Calls": 1, "TotalDurationNs": 1e5, "AverageNs": 1e5, "Percentage": 10},
                {"Name": "kC", "Calls": 4, "TotalDurationNs": 4e6, "AverageNs": 1e6, "Percentage": 5}])
    pf = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = []
    for d in (1, 2):       # kA: two dispatches, each 1e6 FP64 FMA + 5e5 FP32 adds, split over two instances
        for inst in range(2):
            rows.append({"Dispatch_Id": d, "Kernel_Name": "kA", "Counter_Name": "SQ_INSTS_VALU_FMA_F64",
                         "Counter_Value": 5e5})
            rows.append({"Dispatch_Id": d, "Kernel_Name": "kA", "Counter_Name": "SQ_INSTS_VALU_ADD_F32",
                         "Counter_Value": 2.5e5})
    rows.append({"Dispatch_Id": 3, "Kernel_Name": "kB", "Counter_Name": "SQ_INSTS_VALU_TRANS_F32",
                 "Counter_Value": 1e6})
    # kC: 4 calls in the timed run but one dispatch in the counter run (a run of the same command
    # can launch a kernel a different number of times): FLOPs per dispatch x calls
    rows.append({"Dispatch_Id": 4, "Kernel_Name": "kC", "Counter_Name": "SQ_INSTS_VALU_FMA_F32",
                 "Counter_Value": 1e6})
    _write_csv(str(tmp_path / "p" / "r" / "r_counter_collection.csv"), pf, rows)
    bench.summarize_profiles("flops", [str(tmp_path / "s"), str(tmp_path / "p")])
    lines = capsys.readouterr().out.strip().splitlines()
    assert lines[0] == "# source_sha256: " + bench.kernel_source_hash()
    a = [l.split() for l in lines[2:] if l.startswith("kA")][0]
    assert a[1:3] == ["2", "2"]
    # FP64: 2 dispatches x 1e6 FMA x 64 lanes x 2 = 2.56e8 FLOP in 2 ms -> 0.128 TFLOP/s
    assert float(a[5]) == pytest.approx(0.256) and float(a[7]) == pytest.approx(0.128, abs=0.01)
    assert float(a[4]) == pytest.approx(0.064)
    assert float(a[9]) == pytest.approx(0.128e12 / bench.PEAK_FP64_VECTOR, abs=1e-3)
    c = [l.split() for l in lines[2:] if l.startswith("kC")][0]
    # 4 x 1e6 FMA x 64 lanes x 2 = 5.12e8 FLOP in 4 ms -> 0.128 TFLOP/s
    assert c[1:3] == ["4", "1"] and float(c[4]) == pytest.approx(0.512) and float(c[6]) == pytest.approx(0.128, abs=0.01)
    b = [l.split() for l in lines[2:] if l.startswith("kB")][0]
    assert float(b[-1]) == pytest.approx(64e6 / 1e-4 / 1e9)


def test_counter_flops_are_reported_only_for_the_recorded_sources(tmp_path, monkeypatch):
    f = tmp_path / "insts.txt"
    body = "lf::k_maps_tile<false>, 3 dispatches\ncounter FLOPs per dispatch: FP32 7.159e+09, FP64 7.144e+08; algorithmic 4.907e+10\n"
    f.write_text("# header\n# source_sha256: %s\n" % bench.kernel_source_hash() + body)
    monkeypatch.setattr(bench, "INSTS_FILE", str(f))
    assert bench.recorded_counter_flops() == (7.159e9, 7.144e8)
    f.write_text("# source_sha256: 0\n" + body)
    assert bench.recorded_counter_flops() is None
