"""Host logic of the benchmark (no GPU): the algorithmic byte model of the piece kernel, the
counter-traffic summary and its source guard, and the refusal of more than one GPU."""
from __future__ import annotations

import csv
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_heavy_launch_bytes(bench):
    J, m_heavy, npieces = 256, 1000, 10
    dense = {"ran": 1, "sparse": 0, "visits": 700, "light_visits": 200, "merged": 400, "light_merged": 150}
    sparse = dict(dense, sparse=1)
    idle = dict(dense, ran=0)
    # per merged row the head's row, the edge hash and (weighted cascade) the threshold; a
    # sparse launch reads the ids of the edges it visits
    assert bench.heavy_launch_bytes(sparse, J, False, m_heavy, npieces) == 500 * 4 + 250 * J
    assert bench.heavy_launch_bytes(sparse, J, True, m_heavy, npieces) == 500 * 4 + 250 * (J + 4)
    # a dense launch reads every split-row edge id and the piece table instead
    assert bench.heavy_launch_bytes(dense, J, True, m_heavy, npieces) == 250 * (J + 4) + 4 * m_heavy + 20 * npieces
    assert bench.heavy_launch_bytes(idle, J, True, m_heavy, npieces) == 0


def _counter_dir(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_pmc_scales_by_the_copy_calibration(bench, tmp_path):
    heavy = "void hfr::k_sweep_heavy<64, 1, 2>(int const*)"
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = bench.COPY_BYTES / 1024
    # FETCH_SIZE reads half the copied bytes, WRITE_SIZE all of them; values summed per dispatch
    _counter_dir(tmp_path / "F", [
        {"Dispatch_Id": 1, "Kernel_Name": copy, "Counter_Value": gib_kib / 4},
        {"Dispatch_Id": 1, "Kernel_Name": copy, "Counter_Value": gib_kib / 4},
        {"Dispatch_Id": 2, "Kernel_Name": heavy, "Counter_Value": 100.0},
        {"Dispatch_Id": 3, "Kernel_Name": heavy, "Counter_Value": 300.0},
        {"Dispatch_Id": 4, "Kernel_Name": "other", "Counter_Value": 5.0e6},
    ])
    _counter_dir(tmp_path / "W", [
        {"Dispatch_Id": 1, "Kernel_Name": copy, "Counter_Value": gib_kib},
        {"Dispatch_Id": 2, "Kernel_Name": heavy, "Counter_Value": 10.0},
        {"Dispatch_Id": 3, "Kernel_Name": heavy, "Counter_Value": 30.0},
    ])
    text = bench.summarize_pmc(str(tmp_path / "F"), str(tmp_path / "W"), "cmd {counter} {out}")
    kv = dict(line[2:].split(": ", 1) for line in text.splitlines() if line.startswith("- "))
    assert float(kv["fetch_bytes_per_launch"]) == pytest.approx(200.0 * 1024 * 2)
    assert float(kv["write_bytes_per_launch"]) == pytest.approx(20.0 * 1024)
    assert float(kv["traffic_bytes_per_launch"]) == pytest.approx(200.0 * 1024 * 2 + 20.0 * 1024)
    assert kv["source_sha256"].strip("`") == bench.kernel_source_hash()


def test_measured_traffic_requires_the_same_sources(bench, tmp_path, monkeypatch):
    f = tmp_path / "traffic.md"
    f.write_text(f"- traffic_bytes_per_launch: 1234\n- source_sha256: `{bench.kernel_source_hash()}`\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() == 1234.0
    f.write_text("- traffic_bytes_per_launch: 1234\n- source_sha256: `0000`\n")
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
