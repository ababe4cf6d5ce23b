"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline entry,
the counter scaling of the HBM traffic summary, the kernel statistics table
and the hash check that keeps stale traffic counters out of the JSON line.
The profiler outputs are small synthetic CSV files in rocprofv3's columns."""

import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_takes_the_kernel_with_most_device_time():
    launches = ([{"kernel": "prrlu_kernel<2, 6, false, false, 8>", "kind": "prrlu", "us": 700.0, "flops": 3.6e7}] * 4
                + [{"kernel": "contract_kernel<0, false, Tile<32, 32> >", "kind": "contract", "us": 8.0,
                    "flops": 3.0e7}] * 10)
    r = bench.roofline(launches)
    assert r["kernel"] == "prrlu_kernel<2, 6, false, false, 8>"
    assert r["launches"] == 4 and r["bound"] == "alu"
    assert r["avg_launch_us"] == pytest.approx(700.0)
    assert r["achieved"] == pytest.approx(3.6e7 / 700e-6 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["share_of_kernel_time"] == pytest.approx(2800.0 / 2880.0)
    assert r["traffic"] is None


def _counter_dir(tmp_path, name, counter, mine_kib, copy_kib):
    d = tmp_path / name
    d.mkdir()
    rows, i = [], 0
    for v in mine_kib:
        rows.append((i, "void aci::(anonymous namespace)::prrlu_kernel<2, 6, false, false, 8>(aci::PrrluArgs)", v))
        i += 1
    rows.append((i, "void aci::(anonymous namespace)::contract_kernel<0, false, Tile<32, 32> >(aci::ContractArgs)",
                 1e6))
    i += 1
    for v in copy_kib:
        rows.append((i, "void at::native::neg_kernel_cuda(...)", v))
        i += 1
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for di, k, v in rows:
            w.writerow([di, k, counter, v])
    return str(d)


def test_traffic_summary_scales_by_the_calibration_pass(tmp_path):
    calib_kib = bench.CALIB_BYTES / 1024.0
    # FETCH_SIZE reads half of a plain pass, WRITE_SIZE all of it
    fd = _counter_dir(tmp_path, "fetch", "FETCH_SIZE", [600.0, 700.0, 800.0], [calib_kib / 2] * 3)
    wd = _counter_dir(tmp_path, "write", "WRITE_SIZE", [500.0, 500.0], [calib_kib] * 3)
    bj = tmp_path / "bench.json"
    bj.write_text("[bench] log line\n" + json.dumps({"roofline": {"kernel": "prrlu_kernel<2, 6, false, false, 8>"}}))
    out = bench.summarize_pmc(fd, wd, str(bj))
    blob = json.loads(out.split("```json")[1].split("```")[0])
    assert blob["fetch_size_copy_factor"] == pytest.approx(0.5)
    assert blob["write_size_copy_factor"] == pytest.approx(1.0)
    assert blob["fetch_size"] == pytest.approx(700.0 * 1024 / 0.5)
    assert blob["write_size"] == pytest.approx(500.0 * 1024)
    assert blob["traffic"] == pytest.approx(blob["fetch_size"] + blob["write_size"])
    assert blob["source_hash"] == bench.source_hash("prrlu")


def test_stats_table_keeps_the_library_kernels(tmp_path):
    with open(tmp_path / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["void aci::(anonymous namespace)::prrlu_kernel<2, 6, false, false, 8>(aci::PrrluArgs)",
                    10, 7.5e6, 7.5e5, 90, 7.0e5, 8.0e5, 1])
        w.writerow(["void at::native::fill_kernel(...)", 3, 3000, 1000, 1, 900, 1100, 1])
    rows = bench.kernel_stats_table(str(tmp_path))
    assert len(rows) == 3
    assert rows[2] == "| `prrlu_kernel<2, 6, false, false, 8>` | 10 | 7.500 | 750.0 | 700.0 | 800.0 |"


def test_traffic_is_reported_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    k = "prrlu_kernel<2, 6, false, false, 8>"
    good = {"kernel": k, "source_hash": bench.source_hash("prrlu"), "traffic": 123.0}
    (prof / "x_traffic.md").write_text("text\n```json\n" + json.dumps(good) + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash is over the kernel sources, which the temporary root does not hold
    monkeypatch.setattr(bench, "source_hash", lambda kind: good["source_hash"])
    assert bench.measured_traffic(k) == 123.0
    monkeypatch.setattr(bench, "source_hash", lambda kind: "0" * 16)
    assert bench.measured_traffic(k) is None
    assert bench.measured_traffic("prrlu_kernel<1, 6, false, false, 4>") is None
