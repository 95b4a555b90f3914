"""Host-side pieces of bench.py (CPU only, no GPU): the one-GPU guard, the
rocprofv3 counter summary and the stored HBM traffic lookup."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counters_summary_means_per_dispatch(tmp_path, capsys):
    # two dispatches of one kernel, one of another, over two result files
    d = tmp_path / "run" / "host"
    d.mkdir(parents=True)
    head = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    (d / "a_counter_collection.csv").write_text(
        head + '1,"k_push(smf::Geom, smf::State)",FETCH_SIZE,100\n'
               '1,"k_push(smf::Geom, smf::State)",WRITE_SIZE,10\n'
               '2,"k_relabel(smf::Geom)",FETCH_SIZE,7\n')
    (d / "b_counter_collection.csv").write_text(
        head + '3,"k_push(smf::Geom, smf::State)",FETCH_SIZE,300\n'
               '3,"k_push(smf::Geom, smf::State)",WRITE_SIZE,30\n')
    bench.counters_summary(str(tmp_path / "run"))
    rows = [json.loads(line) for line in capsys.readouterr().out.splitlines()]
    assert [r["kernel"] for r in rows] == ["k_push", "k_relabel"]
    assert rows[0]["dispatches"] == 2
    assert rows[0]["per_dispatch"] == {"FETCH_SIZE": 200.0, "WRITE_SIZE": 20.0}
    assert rows[1]["per_dispatch"] == {"FETCH_SIZE": 7.0}


def test_stored_traffic_only_for_the_kernels_it_was_taken_on(monkeypatch):
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    with open(path) as f:
        rec = json.load(f)
    cal = rec["copy_calibration"]
    # the copy kernel reads and writes copy_bytes: the factors turn counter
    # KiB into bytes
    assert cal["fetch_factor"] == pytest.approx(cal["copy_bytes"] / 1024 / cal["FETCH_SIZE_KiB"], rel=1e-3)
    assert cal["write_factor"] == pytest.approx(cal["copy_bytes"] / 1024 / cal["WRITE_SIZE_KiB"], rel=1e-3)
    # bytes per launch = calibrated read bytes + calibrated write bytes (the
    # stored KiB are rounded to 0.1 KiB and the factors to 1e-4: up to about
    # 150 bytes apart)
    for name, k in rec["kernels"].items():
        want = 1024 * (k["FETCH_SIZE_KiB"] * cal["fetch_factor"] + k["WRITE_SIZE_KiB"] * cal["write_factor"])
        assert k["hbm_bytes_per_launch"] == pytest.approx(want, rel=1e-4, abs=160), name
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: rec["kernel_source_sha256"])
    assert bench.stored_traffic("k_bfs_level") == rec["kernels"]["k_bfs_level"]["hbm_bytes_per_launch"]
    assert bench.stored_traffic("no_such_kernel") is None
    # any change of the kernel source voids the stored figures
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 64)
    assert bench.stored_traffic("k_bfs_level") is None
